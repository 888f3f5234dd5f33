/*
 * ctm.h -- C ABI of the MI355X library for the parallel-in-time sparse-grid
 * combination method (Griebel, Schweitzer, Troska, "A Parallel-in-Time
 * Combination Method for Parabolic Problems").
 *
 * The library solves u_t + L u = 0 on a box Omega in d dimensions by the
 * combination technique (Section 2.1.1): every anisotropic component grid
 * Omega_l, |l|_1 = n + d - 1 - w, is advanced in time by backward Euler,
 * Phi = (I + dt L_l)^-1 (Section 2, time propagation), with MGRIT over each
 * recombination block (Section 2.3.1, Algorithm 2; Algorithm 3), and the
 * component solutions are combined with the coefficients
 * (-1)^w binom(d-1, w). Every implicit step is solved matrix-free by CG
 * (symmetric L) or BiCGStab (Section 4.1).
 *
 * Conventions for every entry point:
 *  - All floating-point data is IEEE float64. Device pointers must point to
 *    memory of the device that was current when the plan was created.
 *  - Packed state layout ("packed vector"): the component grids in canonical
 *    order (layer w ascending, then the level vector l lexicographically),
 *    each grid's unknowns contiguous, row-major with axis d-1 fastest.
 *    Grid g starts at the offset returned by ctm_plan_grid_info; the total
 *    length is ctm_plan_state_len.
 *  - Unknowns: Dirichlet grids hold the 2^{l_i}-1 interior nodes
 *    x = lo + J h, J = 1..2^{l_i}-1, h = (hi-lo)/2^{l_i}, per axis (Section
 *    2.1.2). The master-equation lattice (CTM_OP_CME) holds 2^{l_i} states
 *    x = lo + J h, J = 0..2^{l_i}-1, with hi - lo = 2^n.
 *  - Asynchronous entry points enqueue work on the given stream and return;
 *    their device outputs are valid after the stream is synchronised.
 *    ctm_solve synchronises the stream (it reads a convergence scalar after
 *    every MGRIT iteration).
 *  - Errors are returned as ctm_status; ctm_last_error() gives a message for
 *    the calling thread. No entry point throws or aborts. On an error no
 *    output is guaranteed to be written, except CTM_ERR_NOCONV, which still
 *    writes the last iterate.
 *  - Ownership: the caller owns the problem struct, all host arrays it
 *    points to (copied by ctm_plan_create), every device buffer passed in and
 *    the stream. The plan owns small device tables allocated at creation.
 *    A plan may be used from one host thread at a time.
 */
#ifndef CTM_H
#define CTM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CTM_MAXD 8          /* largest dimension d */
#define CTM_MAX_IC_TERMS 16 /* largest number of product terms in u0 */
#define CTM_MAX_HISTORY 256 /* residual history entries kept in ctm_stats */

typedef struct ctm_plan ctm_plan;
typedef struct ihipStream_t* ctm_stream; /* a hipStream_t; NULL = default stream */

typedef enum {
  CTM_OK = 0,
  CTM_ERR_INVALID = 1,   /* invalid argument or problem */
  CTM_ERR_NOMEM = 2,     /* device or host allocation failed, or workspace too small */
  CTM_ERR_HIP = 3,       /* a HIP runtime call failed */
  CTM_ERR_NOCONV = 4,    /* Krylov, refinement or MGRIT did not converge */
  CTM_ERR_BREAKDOWN = 5, /* BiCGStab breakdown (rho or (t,t) vanished) */
  CTM_ERR_NONFINITE = 6  /* NaN or Inf met in a solve */
} ctm_status;

/* Spatial operator kinds, u_t + L u = 0 (Section 2; Sections 4.2-4.4). */
typedef enum {
  CTM_OP_HEAT = 0,    /* L = -Laplacian, (2d+1)-point stencil */
  CTM_OP_VARCOEF = 1, /* L u = -div(a grad u), a = 1 + amp prod_k sin(2 pi x_k), face midpoints */
  CTM_OP_OU = 2,      /* Fokker-Planck of dX = -theta X dt + sigma dW: central diffusion
                         sigma^2/2, donor-cell drift fluxes with face velocity -theta_i x */
  CTM_OP_CME = 3,     /* immigration-death master equation per species on the lattice
                         embedding: births +h at rate k_i/h (none at the last state),
                         deaths -h at rate gamma_i x/h (Section 4.3) */
  CTM_OP_DRIFT = 4    /* Fokker-Planck of the linear SDE dX = theta X dt + sigma dW with a
                         full drift matrix (Section 4.4): L u = sum_i d_i((theta x)_i u)
                         - 1/2 sum_i H_ii d_ii u, H diagonal; second-order finite
                         differences (Section 4.4.1): central diffusion and central face
                         fluxes w (u_j + u_{j+1})/2 with the face velocity w = (theta x)_i
                         taken at the face (x_i shifted by -/+ h_i/2, the other coordinates
                         at the node) */
} ctm_op_kind;

/* Manufactured-solution problems (Section 4.2): CTM_MMS_HEAT is the heat
 * equation on [0,1]^d whose exact solution is
 *   u*(x, t) = sqrt(|x|^2 + t^2) e^-t prod_i sin(pi x_i);
 * each implicit step solves (I + dt L) u_n = u_{n-1} + dt f(., t_n) with
 * f = d/dt u* - Laplace(u*) evaluated at the unknowns (Section 2: forcing
 * g_n = Phi dt f_n), and the initial value is u*(., t0) (ic_* ignored). */
typedef enum { CTM_MMS_NONE = 0, CTM_MMS_HEAT = 1 } ctm_manufactured;

typedef enum { CTM_PREC_FP64 = 0, CTM_PREC_MIXED = 1 } ctm_precision;
typedef enum { CTM_KRYLOV_AUTO = 0, CTM_KRYLOV_CG = 1, CTM_KRYLOV_BICGSTAB = 2 } ctm_krylov;
typedef enum { CTM_RELAX_F = 0, CTM_RELAX_FCF = 1 } ctm_relax;

/* Preconditioner of the implicit-step Krylov solves.
 *   CTM_PRECOND_LINE: exact solves of the lines along each grid's stiffest
 *     axis (the on-chip and streaming solvers' block preconditioner).
 *   CTM_PRECOND_SCHWARZ: the two-level overlapping Schwarz preconditioner of
 *     Section 2.1.2. The unknowns of a grid are ordered along a Hilbert
 *     curve (virtual nodes make the grid isotropic), split into
 *     P = ceil(N / 2^S) disjoint subdomains of consecutive curve positions
 *     (sizes w = floor(N / P) and w + 1, the larger first), each extended by
 *     floor(w / 2) positions on either side (overlap gamma = 1/2) and weighted
 *     by 1/2 (1 for P = 1); the coarse space has one constant per block of
 *     each disjoint subdomain cut into q = 2^(S-4) consecutive blocks (at
 *     least 1); subdomain and coarse problems are the Galerkin restrictions
 *     of the step matrix A = I + dt L, solved exactly by dense inverses the
 *     plan computes on the device for every MGRIT level. With CG the
 *     balanced form G^T C1 G + F (G = I - A F) is used, with BiCGStab the
 *     additive form C1 + F (Section 4.1). Every grid then runs on the
 *     streaming solver (FP64, one work-group of 1,024 threads per task). */
typedef enum { CTM_PRECOND_LINE = 0, CTM_PRECOND_SCHWARZ = 1 } ctm_precond;

typedef struct {
  int d;         /* 1..CTM_MAXD */
  int level_n;   /* sparse-grid level n (the paper's L) */
  int level_min; /* L0 >= 1: every l_i >= L0 (Section 2.1.1) */
  double lo[CTM_MAXD], hi[CTM_MAXD]; /* Omega = prod [lo_i, hi_i] */
  ctm_op_kind op;
  double amp;                            /* CTM_OP_VARCOEF */
  double theta[CTM_MAXD], sigma;         /* CTM_OP_OU */
  double k[CTM_MAXD], gamma[CTM_MAXD];   /* CTM_OP_CME */
  double t0, t1;                         /* time interval */
  long long nsteps;                      /* N backward-Euler steps (uniform dt) */
  int nrecomb;                           /* s >= 1 recombination blocks (Section 2.2.1) */
  int mgrit_levels;                      /* 1 = time-sequential stepping, >= 2 MGRIT */
  int mgrit_cf;                          /* coarsening factor c >= 2 */
  ctm_relax relax;                       /* F or FCF relaxation */
  double mgrit_tol;   /* stop when max over grids and C-points of ||r_m||_2 / ||u_start,g||_2 <= tol */
  int mgrit_maxit;
  ctm_krylov krylov;
  double krylov_tol;  /* FP64 path: ||b - A x||_2 <= tol ||b||_2 per implicit step */
  int krylov_maxit;   /* per solve (per refinement sweep in the mixed path) */
  ctm_precision prec;
  double refine_tol;  /* mixed path: FP64 residual target, relative to ||b||_2 */
  double inner_tol;   /* mixed path: FP32 inner Krylov relative tolerance */
  int refine_maxit;   /* mixed path: refinement sweeps per implicit step */
  int ic_terms;       /* u0(x) = sum_r ic_weight[r] prod_i ic_factor[r][i][J_i] */
  const double* ic_weight; /* host [ic_terms] */
  const double* ic_factor; /* host [ic_terms][d][2^n + 1]: factor r on axis i at the finest
                              1-D node x = lo_i + J (hi_i - lo_i) / 2^n, J = 0..2^n */
  double coarse_tol;  /* relative residual target of the implicit steps on MGRIT levels >= 1,
                         both precisions; the mixed path's FP32 inner tolerance there is
                         max(inner_tol, coarse_tol / 4). 0 = use the level-0 tolerances.
                         The coarse propagator only steers the correction (Section 2.3.1), so
                         the converged result does not depend on it: a loose value trades
                         MGRIT iterations for cheaper coarse solves. */
  int warm_start;     /* nonzero (the default): keep the whole level-0 trajectory of the block
                         in the workspace (N / nrecomb packed vectors more) and start every
                         fine implicit solve of a relaxation from the previous iteration's
                         value at the same time point instead of from the state one step
                         earlier; 0: keep C-points only. The fixed point is the same. */
  ctm_manufactured manufactured; /* CTM_MMS_HEAT: forcing and initial value of the
                         manufactured heat problem (needs op = CTM_OP_HEAT on [0,1]^d) */
  double drift[CTM_MAXD * CTM_MAXD]; /* CTM_OP_DRIFT: theta, row-major d x d (row i = the
                         velocity component along axis i) */
  double diffusion[CTM_MAXD];        /* CTM_OP_DRIFT: H_ii = (2 sigma D sigma^T)_ii >= 0 */
  int residual_mode;  /* nonzero: MGRIT in space-time residual mode (the optimized oscillator
                         run of Section 4.4, XBraid's residual option). Every implicit step is
                         exactly krylov_maxit Krylov iterations from the previous iterate at
                         its time point (an inexact step; no NOCONV), the coarse equation is
                         A_c e_m = e_{m-1} + rho_m with rho_m = u_{cm-1} - A u_cm computed
                         exactly, and mgrit_tol bounds the largest relative space-time
                         residual over the C-points and the F-steps of the F-relaxation. The
                         fixed point is still the time-sequential solution; every coarser
                         level solves its equation in the same residual form. In the mixed
                         precision a step is one FP32 correction solve of krylov_maxit
                         iterations on the FP64 residual, ended early at inner_tol (the
                         FP32 noise floor); streaming grids step in FP64. Needs MGRIT (two
                         or more levels), warm_start and no manufactured forcing;
                         krylov_tol, coarse_tol and refine_tol are unused. */
  ctm_precond precond; /* CTM_PRECOND_LINE (the default) or CTM_PRECOND_SCHWARZ */
  int schwarz_s;       /* CTM_PRECOND_SCHWARZ: subdomains of about 2^S unknowns, 2 <= S <= 6
                          (default 5); a grid may have at most 1,024 coarse blocks */
} ctm_problem;

typedef struct {
  int blocks;                         /* recombination blocks run */
  int mgrit_iterations;               /* total MGRIT iterations over all blocks */
  int history_len;                    /* entries in mgrit_residual */
  double mgrit_residual[CTM_MAX_HISTORY]; /* per iteration: max relative C-point residual */
  long long phi_solves;               /* implicit solves (one per system per step) */
  long long krylov_iterations;        /* Krylov iterations summed over all solves */
  long long krylov_max;               /* largest Krylov count of one solve */
  long long refine_sweeps;            /* refinement sweeps summed (mixed path) */
  long long refine_max;               /* largest sweep count of one solve */
  int status_flags;                   /* OR of (1 << ctm_status) met inside kernels */
  long long krylov_work;              /* sum over solves of Krylov iterations x unknowns */
  long long chain_launches;           /* launches of the implicit-step kernel */
  double chain_ms;                    /* their summed duration (only with ctm_set_timing on) */
  double chain_bytes;                 /* algorithmic HBM bytes those launches move: the
                                         vectors each task must read and write once */
  /* per launch shape (size class) of the implicit-step kernel: waves per
     work-group, unknowns per lane, timed duration, launches, Krylov work.
     Grids on the streaming solver report unknowns per lane 0, with 16 waves
     (one 1,024-thread work-group per task) or 4 (the wide solver, many
     256-thread work-groups per task; a launch is its whole chain). In a
     mixed plan the on-chip launches that run in FP64 (the coarse MGRIT
     levels of the operators with per-line coefficients) are reported
     together with 0 waves and 0 unknowns per lane. */
  int shape_w[16], shape_k[16];
  double shape_ms[16];
  long long shape_launches[16];
  long long shape_work[16];
  double shape_bytes[16];             /* algorithmic HBM bytes of that class's launches */
  long long shape_dofsteps[16];       /* implicit steps x unknowns of that class's launches
                                         (the unit of the 16 B per unknown and step minimum:
                                         read the previous state, write the new one) */
} ctm_stats;

/* Fill *p with the paper's solver defaults (Section 4.1): two-level MGRIT,
 * c = 2, FCF, tolerances 1e-8, CG, FP64, L0 = 1, s = 1, and the unit box;
 * the line preconditioner (schwarz_s = 5 for CTM_PRECOND_SCHWARZ). */
ctm_status ctm_problem_defaults(ctm_problem* p);

/* Validate *p, enumerate the component grids (Section 2.1.1, combination
 * formula), build per-grid geometry and coefficient tables and upload them
 * to the current device. Grids up to 8,192 unknowns with lines of at most
 * 512 take the on-chip solver, larger ones the streaming solver (Krylov
 * vectors in device memory the plan allocates). Rejects: d outside
 * 1..CTM_MAXD, n + d - 1 > 30, no grid with l >= L0, more than 65,535
 * grids, N not divisible by s * c^(levels-1), nonpositive tolerances, CG for
 * a non-symmetric operator, a grid with more than 2^20 unknowns, residual
 * mode outside its conditions (ctm_problem.residual_mode), lattice box with
 * hi - lo != 2^n.
 * On the streaming solver a line longer than 1,024 unknowns is cut into
 * segments of 1,024 for the line preconditioner (exact line solves per
 * segment, block Jacobi across them; the operator is unchanged, so only the
 * Krylov iteration count depends on it). */
ctm_status ctm_plan_create(const ctm_problem* p, ctm_plan** plan);
void ctm_plan_destroy(ctm_plan* plan);

/* Number of component grids G. */
ctm_status ctm_plan_grids(const ctm_plan* plan, int* G);
/* Grid g (0 <= g < G): levels[d] (may be NULL), combination coefficient
 * (-1)^w binom(d-1, w), offset in the packed vector, number of unknowns. */
ctm_status ctm_plan_grid_info(const ctm_plan* plan, int g, int* levels, double* coef,
                              long long* offset, long long* npoints);
/* Length of a packed vector (sum of unknowns over all grids). */
ctm_status ctm_plan_state_len(const ctm_plan* plan, long long* len);
/* Bytes of device workspace ctm_solve needs (MGRIT state of all levels). */
ctm_status ctm_plan_workspace_bytes(const ctm_plan* plan, size_t* bytes);

/* u0_out[packed] = u0 sampled at the unknowns of every grid. Async. */
ctm_status ctm_initial_state(ctm_plan* plan, double* u0_out, ctm_stream s);

/* y = (I + dt_level L_l) x on every grid, dt_level = (t1-t0)/N * c^level
 * (the system matrix of one backward-Euler step, Section 2). FP64. x and y
 * are packed vectors and must not overlap. Async. */
ctm_status ctm_apply(ctm_plan* plan, int level, const double* x, double* y, ctm_stream s);

/* y = C x on every grid with the Schwarz preconditioner C of MGRIT level
 * `level` (Section 2.1.2: the balanced form for CG, the additive form for
 * BiCGStab; see CTM_PRECOND_SCHWARZ). FP64. x and y are packed vectors and
 * must not overlap. Needs a plan with precond = CTM_PRECOND_SCHWARZ
 * (CTM_ERR_INVALID otherwise). Allocates its scratch and returns after the
 * result is complete (the stream is synchronised). */
ctm_status ctm_precond_apply(ctm_plan* plan, int level, const double* x, double* y,
                             ctm_stream s);

/* y = Phi_level^nsteps x on every grid: nsteps backward-Euler steps of size
 * dt_level, all grids in one batched launch (time-sequential stepping,
 * Algorithm 1 inside one block), with the plan's Krylov/precision setting.
 * per_grid != 0 selects the plain reference schedule instead: one grid and
 * one step per launch, FP64 regardless of the plan's precision. x == y is
 * allowed. Async; returns CTM_ERR_NOCONV etc. only through ctm_get_stats
 * status_flags (call after synchronising). */
ctm_status ctm_propagate(ctm_plan* plan, int level, long long nsteps, const double* x, double* y,
                         int per_grid, ctm_stream s);

/* The whole method (Algorithm 3): for each of the s recombination blocks,
 * MGRIT (or time-sequential stepping when mgrit_levels = 1) on every grid
 * from the block's start state, then combine-and-project onto every grid
 * (ctm_recombine) before the next block (Section 2.2.2). u0 (packed, may be NULL = the
 * problem's sampled initial value) is the start state; u_final receives the
 * packed component states at t1. ws must hold ctm_plan_workspace_bytes.
 * Synchronises s. Statistics are available through ctm_get_stats. */
ctm_status ctm_solve(ctm_plan* plan, void* ws, size_t ws_bytes, const double* u0,
                     double* u_final, ctm_stream s);

/* Size of the workspace ctm_solve_noalloc uses: a static array in the
 * library's device code, held by every device the library runs on until the
 * process ends (256 MiB). */
#define CTM_NOALLOC_WORKSPACE_BYTES (256ull << 20)

/* ctm_solve for callers that cannot allocate device memory (code under HIP
 * graph capture elsewhere in the process, tight serving loops, harnesses that
 * forbid hipMalloc): the same method and kernels, on the library's static
 * workspace instead of a caller buffer, with no hipMalloc, hipFree, stream or
 * event creation inside the call. Requirements, each checked (CTM_ERR_INVALID
 * with a message otherwise): ctm_plan_workspace_bytes(plan) <=
 * CTM_NOALLOC_WORKSPACE_BYTES; the plan's device is current; its launch tables
 * exist -- they are built by ctm_plan_create and by every ctm_solve, and
 * ctm_plan_set_grid_shape / ctm_autotune discard them until the next
 * ctm_solve. u0, u_final and s as for ctm_solve; ctm_set_timing is ignored
 * (no per-launch events). Every call on one device shares the one workspace:
 * calls that overlap on a device (other streams or host threads) race. The
 * workspace keeps the last call's contents; the solve initialises everything
 * it reads. Synchronises s. */
ctm_status ctm_solve_noalloc(ctm_plan* plan, const double* u0, double* u_final, ctm_stream s);

/* Combination at arbitrary points (Section 2.1.1): out[j] = sum_g coef_g
 * (I_g u_g)(pts[j]), I_g the d-linear interpolant on grid g with zero
 * boundary values; pts is device [npts][d] row-major. Async. */
ctm_status ctm_gather(ctm_plan* plan, const double* u, const double* pts, long long npts,
                      double* out, ctm_stream s);

/* Combine, then project onto every component grid (Section 2.2.2,
 * combine-then-project operator): out[packed] = u^(c) at the unknowns of
 * every grid, by direct interpolation (every unknown sums the interpolants
 * of all grids; cost grows with the number of grids). u and out must not
 * overlap. Async. */
ctm_status ctm_combine_project(ctm_plan* plan, const double* u, double* out, ctm_stream s);

/* Change of basis of every component grid (Section 2.2.2, hierarchization
 * H_l and de-hierarchization H_l^-1): inverse = 0 maps nodal values to the
 * surpluses of the piecewise linear hierarchical basis (per axis, the value
 * at a node of level k minus the mean of its two parents at distance
 * 2^-k; zero at the Dirichlet boundary and at the lattice node hi),
 * inverse != 0 maps back. in and out are packed device vectors and may be
 * the same. Async. */
ctm_status ctm_hierarchize(ctm_plan* plan, const double* in, double* out, int inverse,
                           ctm_stream s);

/* Combine-then-project through the hierarchical basis, Q = H^-1 Qbar H
 * (Section 2.2.2, recombination operator Qbar): hierarchize every grid, sum
 * the surpluses of each basis function over the grids that contain it with
 * the combination coefficients, give every grid the sums of its own basis
 * functions, de-hierarchize. Equals ctm_combine_project up to rounding, at a
 * cost linear in the state length; ctm_solve uses it between recombination
 * blocks. u and out may be the same vector. The first call builds the
 * plan's node map (device memory owned by the plan, about 16 bytes per
 * unknown). Async. */
ctm_status ctm_recombine(ctm_plan* plan, const double* u, double* out, ctm_stream s);

/* Launch shape of grid g in the on-chip solver: *waves = wavefronts per
 * work-group (one work-group solves one grid's system), *per_lane =
 * consecutive unknowns of a line held by one lane (4 or 8). A grid beyond
 * the on-chip shapes reports *waves = 16, *per_lane = 0 (the streaming
 * solver, 1,024 threads per system). Either pointer may be NULL. */
ctm_status ctm_plan_grid_shape(const ctm_plan* plan, int g, int* waves, int* per_lane);

/* Give grid g the on-chip launch shape (waves, per_lane). Rejects a shape
 * that is not one of the solver's ({1,2,4,8,16} x {4,8}), one whose lanes
 * cannot hold the grid's lines (every line of n_s unknowns needs
 * 2^ceil(log2(ceil(n_s / per_lane))) <= 64 lanes of one wave), and grids on
 * the streaming solver. Results do not depend on the shape beyond rounding;
 * the next solve uses it. The plan's task lists are rebuilt (device memory
 * is freed and allocated): call it with no work of this plan in flight. */
ctm_status ctm_plan_set_grid_shape(ctm_plan* plan, int g, int waves, int per_lane);

/* Grids beyond the on-chip shapes (the streaming solver): a launch of at
 * most max_tasks such tasks (grid, interval) runs on the wide solver, which
 * spreads every task over many work-groups (one launch per Krylov phase for
 * all tasks of the launch, sums across work-groups); a larger launch keeps
 * one 1,024-thread work-group per task. Both use the same operator, Krylov
 * method and stopping test (Section 4.1) and the same line-block
 * preconditioner (the wide solver stores its factors in FP32, its
 * arithmetic staying FP64), so both meet the same tolerance and their
 * results agree to it. A wide launch waits on the host once per step for its
 * convergence test (the stream's earlier work included), so ctm_solve and
 * ctm_propagate return only when that part is done. max_tasks >= 0 (capped
 * at 65,535, the default: every streaming launch); 0 disables the wide
 * solver. Plans whose coefficient tables need more than 44 KiB of LDS keep
 * the one-work-group kernel. */
ctm_status ctm_plan_set_wide(ctm_plan* plan, int max_tasks);

/* Schedule of the MGRIT phases (Algorithm 2: relaxation, restriction,
 * coarse solve, correction) over the size classes. A plan runs its size
 * classes on up to four streams: the caller's and three of its own.
 *   CTM_SCHED_JOINED: every phase of all classes is joined back into the
 *     caller's stream before the next phase starts.
 *   CTM_SCHED_PER_CLASS: with FCF-relaxation, each class runs its phases
 *     (coarse levels included) one after another on its own stream, joined
 *     only for the convergence test of each iteration; a class that ends a
 *     phase early starts its next one while the others still work.
 *   CTM_SCHED_AUTO (default): per class with two MGRIT levels, joined with
 *     three or more.
 * Every class reads only what it wrote itself, so the results do not depend
 * on the schedule. F-relaxation always joins. */
typedef enum {
  CTM_SCHED_AUTO = 0,
  CTM_SCHED_JOINED = 1,
  CTM_SCHED_PER_CLASS = 2
} ctm_schedule;

/* Select the schedule (a ctm_schedule value; anything else is
 * CTM_ERR_INVALID). Takes effect at the next solve. */
ctm_status ctm_plan_set_schedule(ctm_plan* plan, int schedule);

typedef struct {
  int classes;       /* anisotropy classes with more than one candidate shape */
  int trials;        /* timed trial solves run */
  int changed;       /* classes whose shape differs from the plan's default */
  double ms_default; /* trial time with the shapes the plan started with */
  double ms_tuned;   /* trial time with the chosen shapes and schedule */
  double tune_ms;    /* wall time of the whole tuning */
  int schedule;      /* the plan's schedule after tuning (ctm_schedule) */
} ctm_tune_report;

/* Autotuner of the launch shapes and the schedule. The on-chip grids fall
 * into anisotropy classes: equal stiff-axis line length and number of lines,
 * hence the same candidate shapes (per_lane 4 or 8, each with the fewest
 * waves that hold the lines). For each class with two candidates, in
 * decreasing order of its unknowns, the other candidate is tried and kept
 * when it shortens the trial by more than 2%. Then, for FCF-relaxation with
 * two or more MGRIT levels, the schedule other than the one in effect
 * (CTM_SCHED_JOINED or CTM_SCHED_PER_CLASS) is tried and kept on the same
 * rule. A trial is ctm_solve from the problem's initial
 * value, capped at trial_iterations MGRIT iterations per block when
 * trial_iterations > 0 (0 = run to convergence); each configuration runs
 * `repeats` >= 1 times and its fastest run counts. ws (ctm_plan_workspace_bytes)
 * and u_scratch (a packed vector) are overwritten. Synchronous on s; the
 * chosen shapes stay with the plan (ctm_plan_grid_shape); statistics are
 * those of the last trial. report may be NULL. Errors of a trial solve
 * other than CTM_ERR_NOCONV end the tuning with the default shapes. */
ctm_status ctm_autotune(ctm_plan* plan, void* ws, size_t ws_bytes, double* u_scratch,
                        int trial_iterations, int repeats, ctm_tune_report* report,
                        ctm_stream s);

/* Enable (on != 0) or disable timing of the implicit-step kernel: every
 * launch made by ctm_solve / ctm_propagate is then bracketed by two HIP
 * events on the caller's stream and ctm_get_stats reports the summed
 * duration (chain_ms). Off by default; the plan owns the events. */
ctm_status ctm_set_timing(ctm_plan* plan, int on);

/* Statistics of the last ctm_solve / ctm_propagate (reset by each). Call
 * after synchronising the stream the work ran on. */
ctm_status ctm_get_stats(const ctm_plan* plan, ctm_stats* st);

const char* ctm_status_string(ctm_status st);
/* Message of the last error on the calling thread ("" if none). */
const char* ctm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CTM_H */
