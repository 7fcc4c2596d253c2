/*
 * oracle.h -- plain, slow FP64 CPU oracle of the fully discrete time-periodic
 * adjoint method (Zahr, Persson, Wilkening, arXiv:1512.00616).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The product path
 * (the HIP library under paper_1512_00616_amd/) never calls it and shares no
 * source with it.
 *
 * Everything is computed in double precision (double complex where a
 * complex-step derivative is taken).  Derivatives are complex-step
 * derivatives of the residual itself (step 1e-30), i.e. the definition of the
 * Jacobian, not a hand-derived formula.
 *
 * State ordering: u[(K*np + a)*4 + m]  (element K, node a, conserved variable
 * m), the reference-domain state U_X of the ALE formulation (Sec. 4, eqs.
 * ns-cons-ref / transform1-nogcl).
 *
 * Jacobian block layout ("BSR, fixed width 4"): blk[((K*4 + s)*b + row)*b + col]
 * with b = 4*np; slot s = 0 is the diagonal block, slot 1+f the block coupling
 * row element K to its neighbour across local face f (zero block when the face
 * is on the boundary).
 *
 * Stage indexing: stage (n, i) with n = 1..Nt and i = 1..3 is the DIRK stage
 * at t = (n-1+c_i) dt (Sec. 2.1, eq. dirk).  (n, i) = (0, 0) means t = 0.
 *
 * Errors: functions returning int return 0 on success and a negative code on
 * failure (-1 bad argument, -2 no convergence, -3 NaN/Inf, -4 state error);
 * pao_last_error() gives the message.
 */
#ifndef PAO_ORACLE_H
#define PAO_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pao_config {
    int32_t Nr, Nth, p, Nt;         /* O-grid radial x angular quads, degree, steps/period */
    double  r_far, stretch;         /* far-field radius (10), base ratio (1.3 at Nr = 8) */
    double  mach, re, gamma, pr;    /* free stream */
    double  T;                      /* period */
    double  r_blend0, r_blend1;     /* blend radii of the mesh motion (2, 8) */
    int32_t wall_is_farfield;       /* 1: body boundary treated as far field (GCL test) */
    int32_t lin_solver;             /* 0: dense LU, 1: block-Jacobi GMRES */
    int32_t gmres_restart;          /* restart length of the stage GMRES */
    double  lin_rtol;               /* stage linear solve relative tolerance */
    double  newton_atol;            /* stage Newton absolute tolerance on ||R||_2 */
    int32_t newton_maxit;
    int32_t nthreads;               /* OpenMP threads (0 = default) */
} pao_config;

typedef struct pao_ctx pao_ctx;

void        pao_default_config(pao_config* c);
pao_ctx*    pao_create(const pao_config* cfg);
void        pao_destroy(pao_ctx* c);
const char* pao_last_error(const pao_ctx* c);

int64_t pao_num_dofs(const pao_ctx* c);
int32_t pao_num_elems(const pao_ctx* c);
int32_t pao_block_size(const pao_ctx* c);
/* mesh: elem_vert[Ne*3], elem_nbr[Ne*3] (-1 wall, -2 far field), twin[Ne*3],
 * vert_xy[(Nr+1)*Nth*2]; any pointer may be NULL */
void    pao_get_mesh(const pao_ctx* c, int32_t* elem_vert, int32_t* elem_nbr,
                     int8_t* twin, double* vert_xy);
/* element node coordinates X [Ne*np*2] and element areas [Ne] */
void    pao_get_nodes(const pao_ctx* c, double* xnodes, double* area);
/* reference tables for tests: vol points [nq*2], weights [nq], basis at the
 * points [nq*np], mass matrix of the reference triangle [np*np] */
int32_t pao_num_vol_points(const pao_ctx* c);
void    pao_ref_tables(const pao_ctx* c, double* xq, double* wq, double* phiq,
                       double* mhat);
void    pao_dirk_tableau(double A[9], double b[3], double cc[3]);

/* kinematic parameters mu = (h0, theta0 [rad], phi [rad]); recomputes the
 * GCL field gbar for every stage of the period */
int     pao_set_params(pao_ctx* c, const double mu[3]);
/* gbar at stage (n, i), [Ne*np] */
int     pao_gbar(pao_ctx* c, int32_t n, int32_t i, double* out);
/* GCL right-hand side r_g at stage (n, i) [Ne*np] */
int     pao_gcl_rhs(pao_ctx* c, int32_t n, int32_t i, double* out);
/* free stream u = gbar(0) U_inf, plus an optional perturbation */
int     pao_freestream(pao_ctx* c, const double* perturb, double* u);   /* -1 before set_params */
/* mass-matrix product y = M x */
void    pao_mass_apply(const pao_ctx* c, const double* x, double* y);

/* semi-discrete residual r(u, mu, t) at stage (n, i) */
int     pao_residual(pao_ctx* c, int32_t n, int32_t i, const double* u, double* r);
/* Jacobian dr/du at stage (n, i) in BSR layout [Ne*4*b*b] (complex step) */
int     pao_jacobian(pao_ctx* c, int32_t n, int32_t i, const double* u, double* blk);
/* dr/dmu_k at stage (n, i), out[3*Nu] (complex step through map and gbar) */
int     pao_dr_dmu(pao_ctx* c, int32_t n, int32_t i, const double* u, double* out);
/* instantaneous QoIs f = (P^h, F_x^h) at stage (n,i); their u- and
 * mu-derivatives (any output may be NULL) */
int     pao_qoi(pao_ctx* c, int32_t n, int32_t i, const double* u, double f[2],
                double* dfdu /*[2*Nu]*/, double* dfdmu /*[6]*/);

/* BSR helpers */
void    pao_bsr_apply(const pao_ctx* c, const double* blk, int32_t transpose,
                      const double* x, double* y);
/* solve (M - a_dt J) x = rhs (transpose != 0: the transposed operator) with
 * the configured linear solver; returns iterations used */
int     pao_stage_solve(pao_ctx* c, const double* Jblk, double a_dt,
                        int32_t transpose, const double* rhs, double* x);

/* one primal period from u0: fills the trajectory, returns u^(Nt), the time
 * averaged QoIs and ||u^(Nt) - u0||_2 */
int     pao_primal_period(pao_ctx* c, const double* u0, double* uNt,
                          double qoi[2], double* res);
/* tangent sweep about the stored trajectory: out = Phi v (+ mu_k forcing if
 * mu_dir >= 0); dqoi (may be NULL) receives the QoI tangent [2] */
int     pao_tangent_sweep(pao_ctx* c, const double* v, int32_t mu_dir,
                          double* out, double* dqoi);
/* backward adjoint sweep from lambda^(Nt) = lamNt: lam0 = lambda^(0); forced
 * by QoI q when forced_qoi >= 0 (then grad[3] gets the gradient sum of eq.
 * funcl-grad-nosens-dirk, with the explicit term) */
int     pao_adjoint_sweep(pao_ctx* c, const double* lamNt, int32_t forced_qoi,
                          double* lam0, double* grad);

typedef struct pao_krylov_report {
    int32_t outer_its;        /* Newton iterations (shoot) or 1 (adjoint) */
    int32_t krylov_its;       /* total Krylov iterations */
    int32_t sweeps;           /* period sweeps performed */
    double  final_res;        /* final residual norm */
} pao_krylov_report;

/* Newton-Krylov shooting (Alg. 2 with J = Phi - I): u0 in/out */
int     pao_shoot(pao_ctx* c, double* u0, double tol, double eta, int32_t maxit,
                  int32_t max_krylov, pao_krylov_report* rep);
/* periodic adjoint (Alg. 3) about the stored (periodic) trajectory for QoI q:
 * lamNt out [Nu], grad [3] */
int     pao_periodic_adjoint(pao_ctx* c, int32_t q, double rtol, int32_t max_krylov,
                             double* lamNt, double* grad, pao_krylov_report* rep);
/* direct (tangent) gradient of both QoIs on the periodic manifold: dJ[2*3] */
int     pao_tangent_gradient(pao_ctx* c, double rtol, int32_t max_krylov, double* dJ);

/* trajectory access: stage state u_i^(n) (which = 0), stage k_i^(n) (which = 1)
 * or step state u^(n) (which = 2, i ignored) */
int     pao_traj(pao_ctx* c, int32_t which, int32_t n, int32_t i, double* out);
/* stored Jacobian of stage (n, i) */
int     pao_traj_jacobian(pao_ctx* c, int32_t n, int32_t i, double* blk);
/* Pointwise fluxes with this context's gas constants, for closed-form pins
 * (real arguments):
 *   pao_flux_vis: viscous flux F[m][d] (F[2*m + d]) of the state U[4] and its
 *     physical gradient dU[m][d] (dU[2*m + d]); heat = 0 drops the heat flux;
 *   pao_flux_h:   H(U) = F_inv(U) n - U (v_G . n) for a unit normal n, vn = v_G . n;
 *   pao_flux_lf:  the interior numerical flux Fhat(UL, UR, n, vn). */
void    pao_flux_vis(const pao_ctx* c, const double U[4], const double dU[8], int32_t heat, double F[8]);
void    pao_flux_h(const pao_ctx* c, const double U[4], const double n[2], double vn, double H[4]);
void    pao_flux_lf(const pao_ctx* c, const double UL[4], const double UR[4], const double n[2], double vn,
                    double F[4]);
/* Lifting of the interior face f of element K at stage (n, i) for the state
 * u: nodal coefficients lift[(a*4 + m)*2 + D] on the element that carries it
 * (the lower-index side L).  Returns 1 if that is K, 0 if it is the
 * neighbour, a negative code for a boundary face or a bad argument. */
int     pao_face_lift(pao_ctx* c, int32_t n, int32_t i, const double* u, int32_t K, int32_t f, double* lift);

/* counters: total Newton iterations and linear iterations of the last sweep */
void    pao_counters(const pao_ctx* c, int64_t* newton, int64_t* linear);

#ifdef __cplusplus
}
#endif
#endif
