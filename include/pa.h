/*
 * pa.h -- C ABI of the MI355X periodic-adjoint library (libpa.so).
 *
 * The library computes time-periodic solutions of a DG discretisation of the
 * 2-D compressible Navier-Stokes equations on a deforming domain, and the
 * gradients of time-averaged quantities of interest on the manifold of
 * periodic solutions, with the fully discrete adjoint method of Zahr, Persson
 * and Wilkening (arXiv:1512.00616).  The calls follow the paper's statement
 * of the problem (Alg. 4): set the mesh and the kinematic parameters mu, run
 * the primal period, shoot to periodicity, return the QoIs and dJ/dmu.
 *
 * Conventions
 *  - All integers are fixed width; all floating point is IEEE double.
 *  - Host pointers: every array argument of this header is HOST memory owned
 *    by the caller; the library copies in or out synchronously and keeps no
 *    pointer after the call returns.  Device memory is owned by the context.
 *  - State ordering: u[(K*np + a)*4 + m], element K, node a of the element's
 *    equispaced nodal set (t outer, s inner), conserved variable m of the
 *    reference-domain state U_X (Sec. 4 eq. transform1-nogcl with gbar).
 *  - Block layout of dr/du: blk[((K*4 + s)*b + row)*b + col], b = 4*np, slot
 *    s = 0 the diagonal block, s = 1 + f the block coupling element K to its
 *    neighbour across local face f (zero where f lies on the boundary).
 *  - Stage (n, i), n = 1..Nt, i = 1..3 is the DIRK stage at
 *    t = (n - 1 + c_i) dt (Sec. 2.1 eq. dirk); (0, 0) means t = 0.
 *  - Errors: every call returns pa_status; no exception crosses the ABI.
 *    pa_last_error() describes the last failure.  After PA_EDEVICE the
 *    context must be destroyed; after any other error it stays usable.
 *  - Threading: one context per host thread; contexts share nothing.
 */
#ifndef PA_H
#define PA_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum pa_status {
    PA_OK = 0,
    PA_EINVAL = -1,     /* bad argument */
    PA_ENOMEM = -2,     /* device allocation failed */
    PA_EDEVICE = -3,    /* HIP runtime error */
    PA_ENOCONV = -4,    /* Newton / Krylov iteration did not converge */
    PA_ENUMERIC = -5,   /* NaN or Inf, or a singular block */
    PA_ESTATE = -6      /* call out of order (no parameters, no trajectory) */
} pa_status;

typedef struct pa_ctx pa_ctx;

typedef struct pa_config {
    int32_t Nr, Nth;            /* O-grid: radial x angular quads (2 triangles each) */
    int32_t p;                  /* DG polynomial degree, 1..3 */
    int32_t Nt;                 /* DIRK steps per period */
    double  r_far;              /* far-field radius (body radius 1) */
    double  stretch;            /* radial growth ratio at Nr = 8 (refines as stretch^(8/Nr)) */
    double  mach, re, gamma, pr;
    double  T;                  /* period */
    double  r_blend0, r_blend1; /* mesh motion rigid inside r_blend0, at rest beyond r_blend1 */
    int32_t wall_is_farfield;   /* 1: treat the body boundary as far field (GCL checks) */
    int32_t gmres_restart;      /* stage GMRES restart length (<= 64) */
    double  lin_rtol;           /* stage linear solve relative tolerance */
    double  newton_atol;        /* stage Newton tolerance on ||M k - dt r||_2 */
    int32_t newton_maxit;
    int32_t max_krylov;         /* outer Krylov basis size (shooting, periodic adjoint) */
    int32_t device;             /* HIP device ordinal */
    int32_t precision;          /* stage solves: PA_PREC_FP64, PA_PREC_FP32 or PA_PREC_BF16 */
    int32_t autotune;           /* 1: time the forward-apply tile shapes on the first stored operator and
                                   keep the fastest (results may then differ from run to run in the last
                                   bits); 0: fixed shape (default) */
    int32_t block_krylov;       /* outer solves with several right-hand sides (the two QoIs' periodic
                                   adjoints, the three parameter tangents of the direct gradient; Sec.
                                   3.2: the matrix is fixed, only the right-hand side changes): 1: one
                                   block Krylov space shared by all (block GMRES; falls back to 0 when the
                                   right-hand sides or a new block are numerically dependent); 0: one
                                   space per system, advanced in lockstep through the same sweeps
                                   (default) */
    /* Stream and device memory (for a host framework such as PyTorch that
     * owns both).  stream: a hipStream_t on which the context enqueues all
     * its device work, in order; NULL: the context creates its own
     * non-blocking stream.  A caller's stream is never destroyed by the
     * library, and every call that returns host results waits for it.
     * dev_alloc / dev_free: when both are set, every device buffer of the
     * context (trajectory checkpoints, Krylov bases, warm-start model and
     * work storage) is obtained as dev_alloc(bytes, user), which returns
     * device memory of at least that size, 256-byte aligned, or NULL on
     * failure (the call then fails with PA_ENOMEM), and released with
     * dev_free(ptr, user) by pa_destroy or when the buffer is dropped;
     * otherwise hipMalloc / hipFree.  The callbacks are called on the host
     * thread that calls into the context. */
    void*   stream;
    void* (*dev_alloc)(uint64_t bytes, void* user);
    void  (*dev_free)(void* ptr, void* user);
    void*   user;
    /* FP64 stage solves of small meshes (N_u <= 16384, gmres_restart <= 64)
     * as one kernel per solve: the whole restarted GMRES of each system in
     * one workgroup, with no launch per iteration (the same algorithm and
     * stopping test as the multi-kernel solve; sums in another fixed order).
     * 0 (default): never; 1: always (PA_EINVAL at pa_create when the mesh is
     * too large); -1: whenever the mesh is small enough.  One workgroup
     * streams the operator through one compute unit, so this pays only where
     * a solve's data is far smaller than the launch cost of its iterations
     * (on the 8x24 p=1 mesh it is about 3x slower than the multi-kernel
     * solve). */
    int32_t wg_solve;
    /* 1: every stage solve of a tangent or adjoint sweep starts from the
     * same stage's solution at the neighbouring step already swept (the
     * previous step forward, the next one backward), kept when its residual
     * is below |b|; the stopping test stays lin_rtol |b|.  0 (default): from
     * zero.  Newton corrections always start from zero. */
    int32_t lin_guess;
    /* 1: the FP64 stage-GMRES iterations between two convergence checks
     * (5 iterations of apply, multi-dot and basis update, one or several
     * systems) are captured once per context as HIP graphs and replayed;
     * the applies then read the stage operator's address from a device slot
     * set before each solve.  The same kernels in the same order: results
     * are bitwise equal to graph = 0.  It removes the host's cost per
     * launch, not the kernels' own durations (on the 8x24 p=1 mesh, where
     * the GPU is busy most of the time, it changes the time to gradient by
     * a few percent); the sampled kernel times of pa_kernel_time do not
     * cover replayed launches.  Needs gmres_restart a multiple of 5, FP64
     * precision and wg_solve = 0 (else PA_EINVAL at pa_create), and a
     * stream that can be captured (not the legacy null stream).
     * 0 (default): every launch from the host. */
    int32_t graph;
} pa_config;

/* Precision of the stage linear solves (Sec. 2.1 eq. dirk, each stage's
 * (M - dt a_ii dr/du) or its transpose):
 *   PA_PREC_FP64: GMRES in FP64 on the FP64 operator;
 *   PA_PREC_FP32 / PA_PREC_BF16: iterative refinement -- the residual
 *     b - A y, the update of y, the stopping test (lin_rtol) and everything
 *     outside the linear solves stay FP64; each correction is one GMRES
 *     cycle in FP32 arithmetic on a copy of the block-Jacobi-scaled stage
 *     operator stored in FP32 or BF16.  Converged results agree with the
 *     FP64 mode to the solve tolerance; the copy costs 4 (FP32) or 2 (BF16)
 *     bytes per off-diagonal block entry per stage. */
enum { PA_PREC_FP64 = 0, PA_PREC_FP32 = 1, PA_PREC_BF16 = 2 };

/* defaults: 8x24 O-grid, p = 1, Nt = 20, r_far 10, stretch 1.3, M 0.2,
 * Re 1000, gamma 1.4, Pr 0.72, T 1, blend 2..8, GMRES(30) 1e-10,
 * Newton 1e-10 / 20, outer basis 100, FP64 stage solves */
void pa_default_config(pa_config* cfg);

/* Builds the mesh, the reference tables and every device buffer the method
 * needs (including the on-device trajectory checkpoints of a whole period).
 * *out is NULL on failure. */
pa_status pa_create(const pa_config* cfg, pa_ctx** out);
void      pa_destroy(pa_ctx* ctx);                /* NULL-safe */
const char* pa_last_error(const pa_ctx* ctx);

int64_t pa_num_dofs(const pa_ctx* ctx);
int32_t pa_num_elems(const pa_ctx* ctx);
int32_t pa_block_size(const pa_ctx* ctx);
/* device bytes held by the context */
int64_t pa_device_bytes(const pa_ctx* ctx);

/* mesh connectivity: elem_vert[Ne*3], elem_nbr[Ne*3] (-1 wall, -2 far field),
 * twin[Ne*3] (neighbour's local face, -1 on the boundary), vert_xy[Nv*2];
 * any pointer may be NULL */
pa_status pa_get_mesh(const pa_ctx* ctx, int32_t* elem_vert, int32_t* elem_nbr, int8_t* twin, double* vert_xy);

/* kinematic parameters mu = (h0, theta0 [rad], phi [rad]) of heave
 * h0 sin(2 pi t/T) and pitch theta0 sin(2 pi t/T + phi) (Sec. 4.1 eq.
 * defmap with one Fourier mode).  Recomputes the GCL field gbar and its
 * mu-derivatives for every stage; invalidates the trajectory. */
pa_status pa_set_params(pa_ctx* ctx, const double mu[3]);

/* initial state u0 [Nu] (host) */
pa_status pa_set_state(pa_ctx* ctx, const double* u0, int64_t n);
/* u0 = gbar(0) U_inf (+ perturb[Nu] if not NULL) */
pa_status pa_set_freestream(pa_ctx* ctx, const double* perturb);
/* which = 0: current u0, 1: u^(Nt) of the last primal period */
pa_status pa_get_state(pa_ctx* ctx, int32_t which, double* out, int64_t n);

/* One primal period from u0 (Sec. 2.2 eq. dirk2): Newton per stage, stores
 * the trajectory (u^(n), k_i^(n), u_i^(n), dr/du and the block-Jacobi
 * inverses of every stage) on the device.  qoi[2] = time-averaged
 * (power, x-force); res = ||u^(Nt) - u0||_2.  Either output may be NULL. */
pa_status pa_primal_period(pa_ctx* ctx, double qoi[2], double* res);

typedef struct pa_shoot_report {
    int32_t newton_its;         /* outer Newton iterations */
    int32_t krylov_its;         /* total tangent sweeps used as matvecs */
    int32_t primal_sweeps;
    int32_t stage_newton_its;   /* summed over all primal sweeps */
    int64_t stage_gmres_its;    /* summed over all stage solves */
    double  res0, res;          /* initial and final ||u^(Nt) - u0||_2 */
    double  ms;                 /* wall time */
    /* optional history, caller-owned host buffers of hist_cap entries (any
     * may be NULL; set them before the call, the library keeps the
     * pointers it was given): res_hist[k] = ||u^(Nt) - u0||_2 after Newton
     * step k (k = 0: the start), krylov_hist[k] = tangent sweeps (outer
     * GMRES iterations) of Newton step k + 1, step_hist[k] = the accepted
     * line-search step of Newton step k + 1.  Entries past min(newton_its +
     * 1, hist_cap) (res_hist) or min(newton_its, hist_cap) (the others) are
     * left as they were. */
    double*  res_hist;
    int32_t* krylov_hist;
    double*  step_hist;
    int32_t  hist_cap;
} pa_shoot_report;

/* Newton-Krylov shooting (Alg. 2 with the Jacobian Phi - I of eq. jac-prim)
 * from the current u0 to ||u^(Nt) - u0||_2 <= tol, inexact Newton with
 * relative GMRES forcing eta.  On success u0 is periodic and the stored
 * trajectory belongs to it.  PA_ENOCONV leaves the last iterate and report. */
pa_status pa_shoot(pa_ctx* ctx, double tol, double eta, int32_t maxit, pa_shoot_report* rep);
/* (The Newton step u0 - lam Delta is globalised by backtracking, lam = 1,
 * 1/2, ..., 1/64: a trial is accepted when its primal period succeeds and
 * lowers ||u^(Nt) - u0||_2.) */

/* Fixed-point iteration (Alg. 1) as a warm start: `periods` primal periods
 * with u0 <- u^(Nt)(u0).  res (may be NULL) receives ||u^(Nt) - u0||_2 of
 * the last period.  The stored trajectory is invalidated. */
pa_status pa_fixed_point(pa_ctx* ctx, int32_t periods, double* res);

/* Shooting as the unconstrained minimisation of j(u0) = 1/2 ||u^(Nt)(u0) -
 * u0||_2^2 (Sec. 2.2 eq. opt-obj), the gradient-based alternative to Alg. 1
 * and 2: memory = 0 is steepest descent, memory = 1..32 L-BFGS with that
 * many correction pairs.  Each iterate's gradient costs one backward
 * (adjoint) sweep (eq. uns-disc-adj-dirk started from lam^(Nt) = u^(Nt) -
 * u0, gradient lam^(0) + u0 - u^(Nt)); steps are accepted by backtracking
 * (alpha = 1, 1/2, ..., 1/2^15) on sufficient decrease of j.  Stops at
 * ||u^(Nt) - u0||_2 <= tol.  The report reuses pa_shoot_report:
 * newton_its = iterations, krylov_its = backward sweeps, primal_sweeps,
 * res0 / res.  PA_EINVAL for tol <= 0, memory outside 0..32 or maxit < 0;
 * PA_ENOCONV after maxit iterations or a failed line search, leaving the
 * last accepted iterate (with its trajectory) and the report. */
pa_status pa_shoot_descent(pa_ctx* ctx, double tol, int32_t memory, int32_t maxit, pa_shoot_report* rep);

/* grad[Nu] (may be NULL) = dj/du0 of j(u0) above at the current u0 from its
 * stored trajectory (one backward sweep), *j (may be NULL) = j(u0).
 * PA_ESTATE without a trajectory. */
pa_status pa_periodicity_gradient(pa_ctx* ctx, double* grad, double* j);

/* Floquet multipliers (eigenvalues of the flow-map Jacobian Phi of Sec. 2.3)
 * about the stored trajectory, e.g. a periodic one after pa_shoot: k steps
 * of Arnoldi with tangent sweeps from a seeded random start (splitmix64),
 * then the eigenvalues of the k x k Hessenberg matrix.  re[k], im[k]
 * (host) receive the Ritz values by decreasing modulus; *nritz the number
 * computed (less than k if an invariant subspace was found); *hsub (may be
 * NULL) the last subdiagonal entry.  1 <= k <= max_krylov.  The orbit is
 * linearly stable when every multiplier lies inside the unit circle. */
pa_status pa_floquet(pa_ctx* ctx, int32_t k, uint64_t seed, double* re, double* im, int32_t* nritz, double* hsub);

typedef struct pa_adjoint_report {
    int32_t krylov_its[2];      /* outer GMRES iterations per QoI */
    int32_t sweeps;             /* backward sweeps in total (the two QoIs ride together) */
    int32_t rhs_sweeps;         /* right-hand sides carried, summed over the sweeps */
    int64_t stage_gmres_its;
    double  rel_res[2];
    double  ms;
} pa_adjoint_report;

/* Periodic adjoint (Alg. 3) for both QoIs about the stored periodic
 * trajectory, and the gradient of eq. funcl-grad-nosens-dirk (Alg. 4).
 * qoi[2] (may be NULL), dJdmu[2*3] (QoI-major). */
pa_status pa_adjoint_gradient(pa_ctx* ctx, double rtol, double qoi[2], double dJdmu[6], pa_adjoint_report* rep);

/* Direct (tangent) gradient about the stored periodic trajectory, the
 * dual of pa_adjoint_gradient (Sec. 2.2: eq. dirk-sens-mvp with the
 * parameter forcing dt dr/dmu_k at every stage; the periodic tangent solves
 * (Phi - I) du0_k = -s_k with s_k the forced sweep from zero).  The three
 * parameter tangents ride in the same sweeps.  dJdmu[2*3] (QoI-major),
 * krylov_its[3] (may be NULL) per parameter; rtol is the outer GMRES
 * relative tolerance. */
pa_status pa_tangent_gradient(pa_ctx* ctx, double rtol, double dJdmu[6], int32_t krylov_its[3]);

/* Sweeps about the stored trajectory (host vectors of length Nu):
 * tangent: out = Phi v (eq. dirk-sens-mvp);
 * adjoint: lam0 = lambda^(0) from lambda^(Nt) = lamNt (eq.
 * uns-disc-adj-dirk-sens-mvp when forced_qoi < 0, eq. uns-disc-adj-dirk2
 * forced by QoI forced_qoi otherwise, then grad[3] receives dJ/dmu). */
pa_status pa_tangent_sweep(pa_ctx* ctx, const double* v, double* out);
pa_status pa_adjoint_sweep(pa_ctx* ctx, const double* lamNt, int32_t forced_qoi, double* lam0, double* grad);

/* ---- unit-level entry points for parity checks (host in, host out) ---- */
pa_status pa_dbg_gbar(pa_ctx* ctx, int32_t n, int32_t i, double* out /*[Ne*np]*/);
pa_status pa_dbg_dgbar(pa_ctx* ctx, int32_t n, int32_t i, double* out /*[3*Ne*np]*/);
pa_status pa_dbg_residual(pa_ctx* ctx, int32_t n, int32_t i, const double* u, double* r);
pa_status pa_dbg_jacobian(pa_ctx* ctx, int32_t n, int32_t i, const double* u, double* blk);
pa_status pa_dbg_dr_dmu(pa_ctx* ctx, int32_t n, int32_t i, const double* u, double* out /*[3*Nu]*/);
/* instantaneous QoIs, df/du [2*Nu] and df/dmu [2*3]; outputs may be NULL */
pa_status pa_dbg_qoi(pa_ctx* ctx, int32_t n, int32_t i, const double* u, double f[2], double* dfdu, double* dfdmu);
/* y = alpha M x + beta op(J) x with J given in the block layout above */
pa_status pa_dbg_bsr_apply(pa_ctx* ctx, const double* blk, double alpha, double beta, int32_t transpose,
                           const double* x, double* y);
/* inverses of the diagonal blocks of M - a_dt J: out[Ne*b*b] */
pa_status pa_dbg_blockinv(pa_ctx* ctx, const double* blk, double a_dt, double* out);
/* solve (M - a_dt J) x = rhs (transposed if transpose != 0) with
 * block-Jacobi GMRES; *iters receives the iteration count */
pa_status pa_dbg_stage_solve(pa_ctx* ctx, const double* blk, double a_dt, int32_t transpose, const double* rhs,
                             double* x, int32_t* iters);
/* one forward and backward pass of the warm-start perceptron
 * in -> width -> width -> width -> out (tanh hidden, linear output) on the
 * device with no context: params flat [W1 b1 W2 b2 W3 b3 W4 b4], W_l
 * row-major [out_l][in_l]; X[in][batch], T[out][batch] column-major batches;
 * *loss = mean squared error, grads laid out as params */
pa_status pa_dbg_mlp(int32_t in, int32_t width, int32_t out, int32_t batch, const float* params, const float* X,
                     const float* T, float* loss, float* grads);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the pass
 * of pa_dbg_mlp with every array in DEVICE memory of the current device --
 * params, X, T (inputs) and *loss, grads (outputs), laid out as in
 * pa_dbg_mlp -- enqueued on `stream` (hipStream_t; NULL = the null stream)
 * and not waited for.  The activations and back-propagation buffers live in
 * a fixed work array of PA_MLP_SCRATCH_FLOATS floats per GPU, which the
 * library holds until the process ends; the call allocates nothing.  It
 * needs (3 width + out + 2 max(in, width, out)) batch floats of it and
 * returns PA_EINVAL beyond that.  Calls that overlap on one GPU share the
 * array and race: order them on one stream.  Nothing in the array needs
 * clearing between calls (every entry is written before it is read).
 * pa_last_error(NULL) describes a failure. */
#define PA_MLP_SCRATCH_FLOATS (1 << 20)
pa_status pa_mlp_grad_noalloc(int32_t in, int32_t width, int32_t out, int32_t batch, const float* params,
                              const float* X, const float* T, float* loss, float* grads, void* stream);
/* trajectory: which = 0 stage state u_i^(n), 1 stage k_i^(n), 2 step state u^(n) */
pa_status pa_dbg_traj(pa_ctx* ctx, int32_t which, int32_t n, int32_t i, double* out);
/* Host-only checks of the library's small dense eigen-solvers (no device
 * work, callable without a GPU):
 *   pa_dbg_hess_eig: eigenvalues of the real n x n upper Hessenberg matrix
 *     H (row-major; entries below the subdiagonal are ignored) by complex
 *     shifted QR, the routine pa_floquet applies to its Arnoldi matrix;
 *     re[n], im[n] by decreasing modulus.  PA_ENOCONV if QR does not
 *     converge in 100 n iterations.
 *   pa_dbg_sym_eig: eigenvalues w[n] (descending) and eigenvectors V
 *     (row-major n x n, column k belongs to w[k]) of the symmetric matrix A
 *     by cyclic Jacobi rotations, the routine behind the warm start's POD
 *     basis.
 * PA_EINVAL for n outside 1..1024 or a NULL array; pa_last_error(NULL)
 * describes a failure. */
pa_status pa_dbg_hess_eig(int32_t n, const double* H, double* re, double* im);
pa_status pa_dbg_sym_eig(int32_t n, const double* A, double* w, double* V);

/* ---- periodic-constrained optimisation ---- */
typedef struct pa_opt_opts {
    int32_t obj;                /* QoI minimised (0: time-averaged power, 1: x-force) ... */
    double  obj_sign;           /* ... as obj_sign * J[obj] (-1: minimise the work done on the fluid, -P) */
    int32_t con;                /* QoI constrained to con_value (J[con] = con_value); -1: none */
    double  con_value;
    double  lo[3], hi[3];       /* bounds on mu = (h0, theta0, phi) */
    int32_t maxit;              /* SQP iterations */
    double  tol_kkt;            /* stop: projected gradient of the Lagrangian (inf-norm, variables scaled */
    double  tol_c;              /*   to the box) <= tol_kkt and |J[con] - con_value| <= tol_c */
    double  trust;              /* initial step bound in the scaled variables (0: 0.25) */
    double  shoot_tol, shoot_eta;   /* shooting at every evaluation (pa_shoot) */
    int32_t shoot_maxit;
    double  adj_rtol;           /* periodic adjoint tolerance (pa_adjoint_gradient) */
} pa_opt_opts;

typedef struct pa_opt_report {
    int32_t iterations;         /* SQP iterations (accepted or rejected steps) */
    int32_t shoots, gradients;  /* periodic solves and periodic adjoint gradients */
    int32_t newton_its, tangent_sweeps, adjoint_sweeps;
    int32_t converged;          /* 1: both tolerances met; 2: step vanished at a feasible point; 0: neither */
    double  f, c, kkt, lam;     /* objective, constraint violation, KKT measure, multiplier at the end */
    double  mu[3];
    double  ms;
    /* optional history (caller-owned, hist_cap entries, NULL allowed): mu_hist[3k..3k+2], f_hist[k],
       c_hist[k] after iteration k (k = 0: the start) */
    double* mu_hist;
    double* f_hist;
    double* c_hist;
    int32_t hist_cap;
} pa_opt_report;

/* Optimisation over the manifold of periodic solutions (the generalized
 * reduced-gradient method of Sec. 3.3, eqs. opt:disc0-opt:disc2; the
 * problem of Sec. 4.2 with this library's kinematics): minimise
 * obj_sign J[obj](mu) subject to J[con](mu) = con_value and lo <= mu <= hi,
 * where every evaluation shoots to the periodic orbit at mu (Alg. 2, from
 * the previous orbit; the first from the context's current u0) and every
 * accepted point takes the periodic adjoint gradients of both QoIs (Alg. 3,
 * Alg. 4).  The optimiser is a line-search SQP (three-variable QP steps in
 * a trust box, damped BFGS, l1 merit).  mu: start on input, the last
 * accepted point on output; the context is left at that point's periodic
 * orbit.  PA_EINVAL for bad options or a start outside the box;
 * PA_ENOCONV if shooting fails at the start. */
pa_status pa_optimize(pa_ctx* ctx, const pa_opt_opts* opts, double mu[3], pa_opt_report* rep);
/* Host-only check of the SQP subproblem: minimise g.d + 1/2 d^T B d subject
 * to a.d = -c and lo <= d <= hi (3 variables, B row-major symmetric
 * positive definite); when the equality cannot hold in the box its target
 * is clamped to the nearest attainable value.  *lam receives the equality
 * multiplier (g + B d = lam a + bound multipliers).  PA_ENUMERIC if no
 * solution is found. */
pa_status pa_dbg_qp3(const double B[9], const double g[3], const double a[3], double c, const double lo[3],
                     const double hi[3], double d[3], double* lam);

/* ---- many parameter instances ---- */
typedef struct pa_batch_opts {
    int32_t workers;            /* contexts run concurrently, each with its own host thread and stream */
    int32_t shoot_maxit;        /* Newton-Krylov steps per instance (0: one primal period, no shooting) */
    double  shoot_tol, shoot_eta;
    int32_t allow_unconverged;  /* 1: shooting that stops at shoot_maxit still yields the gradient */
    double  adj_rtol;           /* periodic adjoint relative tolerance */
    int32_t keep_going;         /* 1: an instance whose shooting or adjoint fails gets NaN outputs and the
                                   others go on (device errors still stop the batch) */
} pa_batch_opts;

/* The whole method (Alg. 4) for n independent kinematic parameter vectors
 * mu[n][3] on one mesh/configuration: per instance, free stream start,
 * shooting (Alg. 2), then QoIs and dJ/dmu by the periodic adjoint (Alg. 3).
 * Instances are taken in index order by `workers` contexts that run side by
 * side on the device (one host thread and one stream each), which fills the
 * GPU when one instance's kernels alone do not.  Each context holds the full
 * per-instance trajectory storage (pa_device_bytes of one context).
 * Outputs (host, caller-owned): qoi[n][2], dJdmu[n][6], periodicity[n]
 * (||u^(Nt) - u0||_2 after shooting), states[n][N_u] (the initial state u0
 * after shooting, canonical order), dJdmu_direct[n][6] (the same gradient
 * by the direct method, pa_tangent_gradient: the three parameter tangents
 * in the same forward sweeps, so that an instance carries five right-hand
 * sides -- two adjoint, three tangent); any may be NULL (dJdmu_direct NULL:
 * no tangent sweeps).  Results are the same
 * bits as the same instances run one after another on one context.  On
 * failure the first error is returned and pa_last_error(NULL) reports it. */
pa_status pa_batch_gradients(const pa_config* cfg, int32_t n, const double* mu, const pa_batch_opts* opts,
                             double* qoi, double* dJdmu, double* periodicity, double* states,
                             double* dJdmu_direct);

/* ---- learned warm start ---- */
typedef struct pa_ws_opts {
    int32_t  modes;    /* POD modes kept (at most training states - 1, at most 128) */
    int32_t  width;    /* hidden width of the 3 -> w -> w -> w -> modes perceptron (tanh) */
    int32_t  epochs;   /* full-batch Adam steps */
    float    lr;       /* Adam learning rate */
    uint64_t seed;     /* initial weights (splitmix64, Glorot-uniform) */
} pa_ws_opts;

/* Learned warm start for shooting (a start closer to the periodic orbit cuts
 * Newton-Krylov steps, Sec. 2.2).  Training data: S method-generated periodic
 * initial states (e.g. from pa_batch_gradients, or prolonged from a coarser
 * discretisation with pa_prolong) and the inputs they were computed with,
 * params[S][4] = (h0, theta0, phi, Mach), states[S][N_u] (host).  Each
 * state's own free stream gbar(0) U_inf(Mach) is removed, then the POD of the
 * centred deviations is built on the device (method of snapshots) and a
 * perceptron from the normalised inputs to normalised POD coefficients is
 * trained on the device with FP32 kernels by full-batch Adam on the mean
 * squared error; *final_loss (may be NULL) receives the last training loss.
 * Replaces any previous model.  PA_EINVAL for a non-positive Mach number. */
pa_status pa_ws_train(pa_ctx* ctx, const double* params, const double* states, int32_t S, const pa_ws_opts* opts,
                      double* final_loss);
/* u0 = gbar(0) U_inf + mean deviation + POD modes x the coefficients
 * predicted for (mu[3], this context's Mach number); invalidates the
 * trajectory.  PA_ESTATE without a model. */
pa_status pa_ws_predict(pa_ctx* ctx, const double mu[3]);
/* the trained POD (FP64): mean[N_u] deviation from the free stream, modes
 * [min(kmax, k)][N_u] (orthonormal), eig[min(kmax, k)] the eigenvalues of
 * the snapshots' Gram matrix (descending); *k receives the number of modes
 * kept.  Any output may be NULL.  PA_ESTATE without a model. */
pa_status pa_ws_pod(pa_ctx* ctx, int32_t kmax, double* mean, double* modes, double* eig, int32_t* k);
/* pa_shoot from the predicted state for the current parameters; when the
 * first Newton step fails or does not lower ||u^(Nt) - u0||, shooting starts
 * again from the free stream (*fell_back = 1).  The report sums both runs;
 * its history buffers describe the last one. */
pa_status pa_ws_shoot(pa_ctx* ctx, double tol, double eta, int32_t maxit, pa_shoot_report* rep, int32_t* fell_back);
/* Prolongation for warm starts across discretisations (orbits computed on a
 * coarse O-grid used as snapshots of a finer one): u_fine[N_u of fine]
 * (host) = the coarse DG state u_coarse (host, canonical order of the
 * discretisation `coarse`, which must share r_far and stretch with fine)
 * evaluated at every node of `fine` in the fixed reference domain, from the
 * coarse triangle containing the node.  Host-only work; `fine` provides the
 * node coordinates.  PA_EINVAL for a NULL argument or mismatched grids. */
pa_status pa_prolong(const pa_config* coarse, const double* u_coarse, pa_ctx* fine, double* u_fine);
/* model file (binary, this library's layout); load checks N_u */
pa_status pa_ws_save(pa_ctx* ctx, const char* path);
pa_status pa_ws_load(pa_ctx* ctx, const char* path);

/* ---- measurement ---- */
/* kernel ids for pa_kernel_time */
enum {
    PA_K_SPMV = 0,      /* FP64 stage-operator apply (forward) */
    PA_K_PRECOND = 1,   /* block-diagonal apply */
    PA_K_JACOBIAN = 2,
    PA_K_RESIDUAL = 3,
    PA_K_BLOCKINV = 4,  /* diagonal-block LU/inverse and operator formation */
    PA_K_SPMV_LO = 5,   /* low-precision stage-operator apply (mixed-precision modes) */
    PA_K_SPMV_T = 6,    /* FP64 stage-operator apply, transposed */
    PA_K_SPMV_M = 7,    /* FP64 forward apply carrying several right-hand sides in one launch */
    PA_K_SPMV_TM = 8,   /* FP64 transposed apply carrying several right-hand sides in one launch */
    PA_K_MDOT = 9,      /* stage GMRES: multi-column dot-product partials */
    PA_K_GMUPD = 10,    /* stage GMRES: final sums, Givens update and next basis vector */
    PA_K_COUNT = 11
};
/* when on, every 8th launch of each listed kernel carries a pair of HIP
 * events that the launch itself records (hipExtLaunchKernelGGL) at the
 * kernel's start and end on the library's stream, so a sample is the
 * kernel's execution time without the dispatch latency ahead of it
 * (PA_K_BLOCKINV: from the start of the block-factor kernel to the end of
 * the operator formation that follows it); pa_kernel_time returns the
 * launch count since timing was switched on and the sampled mean duration
 * times that count.  Launches replayed from graphs (pa_config.graph) are
 * not counted. */
pa_status pa_set_timing(pa_ctx* ctx, int32_t on);
pa_status pa_kernel_time(pa_ctx* ctx, int32_t kernel, double* total_ms, int64_t* launches);
/* of those launches, the stage-operator applies (PA_K_SPMV, PA_K_SPMV_T,
 * PA_K_SPMV_LO, PA_K_SPMV_M, PA_K_SPMV_TM) and the FP64 stage-GMRES vector
 * kernels (PA_K_MDOT, PA_K_GMUPD) that returned at once without work: GMRES enqueues several
 * iterations ahead of its host-side convergence check, and an apply whose
 * systems have all converged exits on entry.  Bytes moved by a kernel are
 * its per-launch bytes times (launches - skipped).  0 for other kernels;
 * reset by pa_set_timing.  PA_EINVAL for a bad id or a NULL output. */
pa_status pa_kernel_skipped(pa_ctx* ctx, int32_t kernel, int64_t* skipped);
/* for the FP64 stage-GMRES vector kernels (PA_K_MDOT, PA_K_GMUPD): the
 * number of length-N_u vectors their working launches read or wrote since
 * timing was switched on (iteration j of a cycle: j + 2 in k_mdot_part --
 * the basis columns 0..j and w --, j + 3 in the update, which also writes
 * V_{j+1}); their algorithmic bytes are this count times 8 N_u.  0 for
 * other kernels; reset by pa_set_timing.  PA_EINVAL for a bad id or a NULL
 * output. */
pa_status pa_kernel_vectors(pa_ctx* ctx, int32_t kernel, int64_t* vectors);
/* averaged over reps launches of the preconditioned stage-operator apply
 * y = Ahat x (transposed: Ahat^T x) of the stored first stage, Ahat =
 * (M - dt a_11 J) P^{-1} with P its diagonal blocks (timed with HIP events on
 * the library stream; needs a stored trajectory) */
pa_status pa_bench_spmv(pa_ctx* ctx, int32_t reps, int32_t transpose, double* avg_ms);
/* as pa_bench_spmv for the apply that carries nrhs (1..8) right-hand sides
 * in one launch (the form the lockstep solves of several systems use); the
 * stored blocks are read once per launch for all of them */
pa_status pa_bench_spmv_m(pa_ctx* ctx, int32_t reps, int32_t transpose, int32_t nrhs, double* avg_ms);
/* tile shape of the FP64 forward apply: chunks of 16 bytes per lane task
 * (1, 2 or 4; 0 = built-in default) and, after autotuning, the measured
 * microseconds per launch of each shape (-1: not valid for this block size,
 * 0: not measured) */
pa_status pa_tuning(pa_ctx* ctx, int32_t* fwd_chunks, double fwd_us[3]);
/* as pa_bench_spmv for the FP32/BF16 copy of the operator with FP32 vectors;
 * PA_ESTATE unless the context was created with precision FP32 or BF16 */
pa_status pa_bench_spmv_lo(pa_ctx* ctx, int32_t reps, int32_t transpose, double* avg_ms);
/* averaged over reps device-to-device copies of the first stage's stored
 * operator (*bytes receives the size): a plain copy kernel of known size for
 * calibrating hardware traffic counters.  Overwrites the second stage's
 * operator, so the trajectory is invalidated. */
pa_status pa_bench_copy(pa_ctx* ctx, int32_t reps, double* avg_ms, int64_t* bytes);

#ifdef __cplusplus
}
#endif
#endif
