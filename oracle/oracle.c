/*
 * oracle.c -- plain FP64 CPU oracle of the fully discrete time-periodic
 * adjoint method of Zahr, Persson & Wilkening (arXiv:1512.00616).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the product path.  It shares no
 * source with the HIP library.
 *
 * Written for readability, not speed: every quantity is computed the
 * obvious way, in double complex so that one residual routine serves both
 * the residual and its complex-step derivatives (Jacobian dr/du, dr/dmu,
 * QoI derivatives).  Loops over elements may run under OpenMP with a static
 * schedule; no reduction crosses threads.
 *
 * Paper map (sections and equations of arXiv:1512.00616):
 *   semi-discrete ODE M du/dt = r(u, mu, t), constant M ........ Sec. 2.1, eq. semidisc
 *   s-stage DIRK, stage equations ............................... Sec. 2.1, eqs. dirk, dirk-stage
 *   solver-consistent QoI F(u^(0..Nt), k) ........................ Sec. 2.1, eq. qoi-disc
 *   flow map u0 -> u^(Nt) (primal sweep) ........................ Sec. 2.2, eq. dirk2
 *   R(u0) = u^(Nt) - u0, Jacobian Phi - I ........................ Sec. 2.2, eqs. nlsys, jac-prim
 *   directional sensitivity (tangent sweep) ..................... Sec. 2.2, eq. dirk-sens-mvp
 *   Newton-Krylov shooting ....................................... Sec. 2.2, Alg. 2
 *   DIRK adjoint equations, gradient ............................. Sec. 3.1, eqs. uns-disc-adj-dirk,
 *                                                                   funcl-grad-nosens-dirk
 *   backward adjoint map, periodic adjoint system ................ Sec. 3.2, eqs. uns-disc-adj-dirk2,
 *                                                                   fixedpt-dual, jac-dual
 *   adjoint-sensitivity sweep (matvec of Alg. 3) ................. Sec. 3.2, eq. uns-disc-adj-dirk-sens-mvp
 *   gradient on the periodic manifold ............................ Sec. 3.2, Alg. 3 and Alg. 4
 *   Navier-Stokes, stress, heat flux, ideal gas .................. Sec. 4, eqs. ns1-ns5
 *   ALE transformation to a fixed reference domain ............... Sec. 4, eqs. ns-cons-ref,
 *                                                                   transform1-nogcl, transform2-nogcl
 *   rigid heave/pitch kinematics ................................. Sec. 4.1, eq. defmap
 *   QoIs: power and x-force on the body .......................... Sec. 4, eq. qoi
 *
 * Where the paper delegates a detail to other work (DG fluxes, CDG viscous
 * treatment, GCL modification, boundary conditions, DIRK tableau), the
 * reading implemented here is stated at the routine.
 */
#include "oracle.h"

#include <complex.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define CSTEP 1e-30          /* complex-step size */
#define LF_DELTA 1e-2        /* smoothing of |u.n - v.n| in the Lax-Friedrichs speed */
#define WALL_ETA 10.0        /* wall penalty C11 = WALL_ETA / h */

struct pao_ctx {
    pao_config cfg;
    char err[256];
    int Ne, np, nq, nf, b, Nt, nst;
    int64_t Nu;
    int nv;
    double *vxy;
    int32_t *ev, *enb;
    int8_t *etw;
    double *area, *jit;      /* |K| and J_K^{-T} (row-major 2x2) */
    double *xn;              /* node coordinates X [Ne][np][2] */
    double *wbl;             /* blend weight at nodes [Ne][np] */
    /* reference element */
    double *rn;              /* reference nodes [np][2] */
    int *mx, *my;            /* monomial exponents */
    double *C;               /* inverse Vandermonde [np(k)][np(a)] */
    double *xq, *wq, *phq, *dphq;        /* volume points */
    double *sf, *wf;                     /* 1-D face rule on [0,1] */
    double *phf, *dphf, *phfr, *dphfr;   /* face tables [3][nf][np](x2), s and 1-s */
    double *mh, *mhi;                    /* reference mass matrix and inverse */
    /* physics */
    double gam, muv, pr, Uinf[4];
    /* DIRK */
    double A[3][3], bw[3], cc[3], dt;
    /* parameters and GCL field */
    double mu[3];
    int have_params, have_dgb;
    cplx *gb[4];             /* gbar at every stage: base and 3 complex-step directions */
    /* trajectory */
    double *tu, *tk, *tui, *tJ;
    int have_traj;
    int64_t cnt_newton, cnt_lin;
};

static int fail(pao_ctx* c, int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(c->err, sizeof c->err, fmt, ap);
    va_end(ap);
    return code;
}

/* ------------------------------------------------------------------ */
/* small dense linear algebra                                          */
/* ------------------------------------------------------------------ */

/* LU with partial pivoting, ties resolved to the lowest row index.
 * a is n x n row-major, piv[n].  Returns 0, or -3 for a zero pivot. */
static int lu_factor(int n, double* a, int* piv)
{
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = fabs(a[k * n + k]);
        for (int i = k + 1; i < n; ++i)
            if (fabs(a[i * n + k]) > best) { best = fabs(a[i * n + k]); p = i; }
        piv[k] = p;
        if (best == 0.0) return -3;
        if (p != k)
            for (int j = 0; j < n; ++j) { double t = a[k * n + j]; a[k * n + j] = a[p * n + j]; a[p * n + j] = t; }
        for (int i = k + 1; i < n; ++i) {
            double l = a[i * n + k] / a[k * n + k];
            a[i * n + k] = l;
            for (int j = k + 1; j < n; ++j) a[i * n + j] -= l * a[k * n + j];
        }
    }
    return 0;
}

/* solve (LU) x = b in place (trans = 0) or (LU)^T x = b (trans = 1) */
static void lu_solve(int n, const double* a, const int* piv, double* x, int trans)
{
    if (!trans) {
        for (int k = 0; k < n; ++k) { int p = piv[k]; if (p != k) { double t = x[k]; x[k] = x[p]; x[p] = t; } }
        for (int i = 0; i < n; ++i) { double s = x[i]; for (int j = 0; j < i; ++j) s -= a[i * n + j] * x[j]; x[i] = s; }
        for (int i = n - 1; i >= 0; --i) { double s = x[i]; for (int j = i + 1; j < n; ++j) s -= a[i * n + j] * x[j]; x[i] = s / a[i * n + i]; }
    } else {
        /* A = P^T L U  =>  A^T = U^T L^T P */
        for (int i = 0; i < n; ++i) { double s = x[i]; for (int j = 0; j < i; ++j) s -= a[j * n + i] * x[j]; x[i] = s / a[i * n + i]; }
        for (int i = n - 1; i >= 0; --i) { double s = x[i]; for (int j = i + 1; j < n; ++j) s -= a[j * n + i] * x[j]; x[i] = s; }
        for (int k = n - 1; k >= 0; --k) { int p = piv[k]; if (p != k) { double t = x[k]; x[k] = x[p]; x[p] = t; } }
    }
}

static double dot(int64_t n, const double* x, const double* y)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += x[i] * y[i];
    return s;
}
static double nrm2(int64_t n, const double* x) { return sqrt(dot(n, x, x)); }

/* ------------------------------------------------------------------ */
/* reference element: equispaced nodal Lagrange basis, Gauss rules      */
/* ------------------------------------------------------------------ */

/* n-point Gauss-Legendre rule mapped to [0, 1] (weights sum to 1); nodes by
 * Newton iteration on the Legendre polynomial P_n. */
static void gauss01(int n, double* x, double* w)
{
    for (int i = 0; i < n; ++i) {
        double z = cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int j = 2; j <= n; ++j) { double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j; p0 = p1; p1 = p2; }
            if (n == 1) { p1 = z; p0 = 1.0; }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        {   /* final derivative at the converged node */
            double p0 = 1.0, p1 = z;
            for (int j = 2; j <= n; ++j) { double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j; p0 = p1; p1 = p2; }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
        }
        x[n - 1 - i] = 0.5 * (1.0 + z);
        w[n - 1 - i] = 1.0 / ((1.0 - z * z) * dp * dp);   /* = (2/((1-z^2)P'^2)) / 2 */
    }
}

static void basis_at(const pao_ctx* c, double xi, double eta, double* phi, double* dphi)
{
    int np = c->np;
    double m[32], mxv[32], myv[32];
    for (int k = 0; k < np; ++k) {
        int a = c->mx[k], b = c->my[k];
        m[k] = pow(xi, a) * pow(eta, b);
        mxv[k] = a ? a * pow(xi, a - 1) * pow(eta, b) : 0.0;
        myv[k] = b ? b * pow(xi, a) * pow(eta, b - 1) : 0.0;
    }
    for (int a = 0; a < np; ++a) {
        double s = 0, sx = 0, sy = 0;
        for (int k = 0; k < np; ++k) { double ck = c->C[k * np + a]; s += ck * m[k]; sx += ck * mxv[k]; sy += ck * myv[k]; }
        if (phi) phi[a] = s;
        if (dphi) { dphi[2 * a] = sx; dphi[2 * a + 1] = sy; }
    }
}

static const double RV[3][2] = { { 0, 0 }, { 1, 0 }, { 0, 1 } };

static int ref_init(pao_ctx* c)
{
    int p = c->cfg.p, np = (p + 1) * (p + 2) / 2;
    c->np = np;
    c->b = 4 * np;
    c->rn = malloc(sizeof(double) * np * 2);
    c->mx = malloc(sizeof(int) * np);
    c->my = malloc(sizeof(int) * np);
    c->C = malloc(sizeof(double) * np * np);
    /* nodes: t outer, s inner, at (s/p, t/p) */
    int a = 0;
    for (int t = 0; t <= p; ++t)
        for (int s = 0; s <= p - t; ++s) { c->rn[2 * a] = (double)s / p; c->rn[2 * a + 1] = (double)t / p; ++a; }
    int k = 0;
    for (int d = 0; d <= p; ++d)
        for (int j = 0; j <= d; ++j) { c->mx[k] = d - j; c->my[k] = j; ++k; }
    /* V[b][k] = m_k(node_b);  C = V^{-1} by solving V C = I column by column */
    double* V = malloc(sizeof(double) * np * np);
    int* piv = malloc(sizeof(int) * np);
    for (int bb = 0; bb < np; ++bb)
        for (int kk = 0; kk < np; ++kk) V[bb * np + kk] = pow(c->rn[2 * bb], c->mx[kk]) * pow(c->rn[2 * bb + 1], c->my[kk]);
    if (lu_factor(np, V, piv)) { free(V); free(piv); return -1; }
    double* col = malloc(sizeof(double) * np);
    for (int aa = 0; aa < np; ++aa) {
        for (int i = 0; i < np; ++i) col[i] = (i == aa);
        lu_solve(np, V, piv, col, 0);
        for (int kk = 0; kk < np; ++kk) c->C[kk * np + aa] = col[kk];
    }
    free(col); free(V); free(piv);
    /* volume rule: collapsed Gauss, (p+2)^2 points, xi = u(1-v), eta = v */
    int ng = p + 2;
    double *gx = malloc(sizeof(double) * ng), *gw = malloc(sizeof(double) * ng);
    gauss01(ng, gx, gw);
    c->nq = ng * ng;
    c->xq = malloc(sizeof(double) * c->nq * 2);
    c->wq = malloc(sizeof(double) * c->nq);
    int q = 0;
    for (int l = 0; l < ng; ++l)
        for (int kq = 0; kq < ng; ++kq) {
            c->xq[2 * q] = gx[kq] * (1.0 - gx[l]);
            c->xq[2 * q + 1] = gx[l];
            c->wq[q] = gw[kq] * gw[l] * (1.0 - gx[l]);
            ++q;
        }
    c->phq = malloc(sizeof(double) * c->nq * np);
    c->dphq = malloc(sizeof(double) * c->nq * np * 2);
    for (q = 0; q < c->nq; ++q) basis_at(c, c->xq[2 * q], c->xq[2 * q + 1], c->phq + q * np, c->dphq + q * np * 2);
    /* face rule: p+2 Gauss points on [0,1] */
    c->nf = ng;
    c->sf = gx;
    c->wf = gw;
    c->phf = malloc(sizeof(double) * 3 * ng * np);
    c->dphf = malloc(sizeof(double) * 3 * ng * np * 2);
    c->phfr = malloc(sizeof(double) * 3 * ng * np);
    c->dphfr = malloc(sizeof(double) * 3 * ng * np * 2);
    for (int f = 0; f < 3; ++f) {
        const double* r0 = RV[f];
        const double* r1 = RV[(f + 1) % 3];
        for (int j = 0; j < ng; ++j) {
            double s = gx[j], sr = 1.0 - gx[j];
            basis_at(c, r0[0] + s * (r1[0] - r0[0]), r0[1] + s * (r1[1] - r0[1]),
                     c->phf + (f * ng + j) * np, c->dphf + (f * ng + j) * np * 2);
            basis_at(c, r0[0] + sr * (r1[0] - r0[0]), r0[1] + sr * (r1[1] - r0[1]),
                     c->phfr + (f * ng + j) * np, c->dphfr + (f * ng + j) * np * 2);
        }
    }
    /* reference mass matrix (triangle of area 1/2) */
    c->mh = calloc((size_t)np * np, sizeof(double));
    c->mhi = malloc(sizeof(double) * np * np);
    for (q = 0; q < c->nq; ++q)
        for (int i = 0; i < np; ++i)
            for (int j = 0; j < np; ++j) c->mh[i * np + j] += c->wq[q] * c->phq[q * np + i] * c->phq[q * np + j];
    double* t = malloc(sizeof(double) * np * np);
    int* pv = malloc(sizeof(int) * np);
    memcpy(t, c->mh, sizeof(double) * np * np);
    lu_factor(np, t, pv);
    double* e = malloc(sizeof(double) * np);
    for (int aa = 0; aa < np; ++aa) {
        for (int i = 0; i < np; ++i) e[i] = (i == aa);
        lu_solve(np, t, pv, e, 0);
        for (int i = 0; i < np; ++i) c->mhi[i * np + aa] = e[i];
    }
    free(e); free(t); free(pv);
    return 0;
}

/* ------------------------------------------------------------------ */
/* mesh: O-grid around the unit circle, quads split into two triangles  */
/* ------------------------------------------------------------------ */
static void mesh_init(pao_ctx* c)
{
    int Nr = c->cfg.Nr, Nth = c->cfg.Nth, p = c->cfg.p, np = c->np;
    c->nv = (Nr + 1) * Nth;
    c->Ne = 2 * Nr * Nth;
    c->vxy = malloc(sizeof(double) * c->nv * 2);
    double q = pow(c->cfg.stretch, 8.0 / Nr);
    for (int i = 0; i <= Nr; ++i) {
        double r = 1.0 + (c->cfg.r_far - 1.0) * (pow(q, i) - 1.0) / (pow(q, Nr) - 1.0);
        for (int j = 0; j < Nth; ++j) {
            double th = 2.0 * M_PI * j / Nth;
            c->vxy[2 * (i * Nth + j)] = r * cos(th);
            c->vxy[2 * (i * Nth + j) + 1] = r * sin(th);
        }
    }
    int Ne = c->Ne;
    c->ev = malloc(sizeof(int32_t) * Ne * 3);
    c->enb = malloc(sizeof(int32_t) * Ne * 3);
    c->etw = malloc(sizeof(int8_t) * Ne * 3);
#define VID(i, j) ((i) * Nth + (((j) % Nth + Nth) % Nth))
#define EA(i, j) (2 * ((i) * Nth + (((j) % Nth + Nth) % Nth)))
    for (int i = 0; i < Nr; ++i)
        for (int j = 0; j < Nth; ++j) {
            int A = EA(i, j), B = A + 1;
            int va = VID(i, j), vb = VID(i + 1, j), vc = VID(i + 1, j + 1), vd = VID(i, j + 1);
            c->ev[3 * A] = va; c->ev[3 * A + 1] = vb; c->ev[3 * A + 2] = vc;
            c->ev[3 * B] = va; c->ev[3 * B + 1] = vc; c->ev[3 * B + 2] = vd;
            /* A: f0 <-> B(i,j-1).f1 ; f1 <-> B(i+1,j).f2 or far field ; f2 <-> B(i,j).f0 */
            c->enb[3 * A] = EA(i, j - 1) + 1;  c->etw[3 * A] = 1;
            if (i == Nr - 1) { c->enb[3 * A + 1] = -2; c->etw[3 * A + 1] = -1; }
            else { c->enb[3 * A + 1] = EA(i + 1, j) + 1; c->etw[3 * A + 1] = 2; }
            c->enb[3 * A + 2] = B; c->etw[3 * A + 2] = 0;
            /* B: f0 <-> A(i,j).f2 ; f1 <-> A(i,j+1).f0 ; f2 <-> A(i-1,j).f1 or wall */
            c->enb[3 * B] = A; c->etw[3 * B] = 2;
            c->enb[3 * B + 1] = EA(i, j + 1); c->etw[3 * B + 1] = 0;
            if (i == 0) { c->enb[3 * B + 2] = -1; c->etw[3 * B + 2] = -1; }
            else { c->enb[3 * B + 2] = EA(i - 1, j); c->etw[3 * B + 2] = 1; }
        }
#undef VID
#undef EA
    c->area = malloc(sizeof(double) * Ne);
    c->jit = malloc(sizeof(double) * Ne * 4);
    c->xn = malloc(sizeof(double) * Ne * np * 2);
    c->wbl = malloc(sizeof(double) * Ne * np);
    for (int K = 0; K < Ne; ++K) {
        const double* v0 = c->vxy + 2 * c->ev[3 * K];
        const double* v1 = c->vxy + 2 * c->ev[3 * K + 1];
        const double* v2 = c->vxy + 2 * c->ev[3 * K + 2];
        double a = v1[0] - v0[0], bb = v2[0] - v0[0], cc = v1[1] - v0[1], d = v2[1] - v0[1];
        double det = a * d - bb * cc;
        c->area[K] = 0.5 * det;
        c->jit[4 * K] = d / det;   c->jit[4 * K + 1] = -cc / det;
        c->jit[4 * K + 2] = -bb / det; c->jit[4 * K + 3] = a / det;
        int aa = 0;
        for (int t = 0; t <= p; ++t)
            for (int s = 0; s <= p - t; ++s) {
                double X = v0[0] + ((double)s / p) * (v1[0] - v0[0]) + ((double)t / p) * (v2[0] - v0[0]);
                double Y = v0[1] + ((double)s / p) * (v1[1] - v0[1]) + ((double)t / p) * (v2[1] - v0[1]);
                c->xn[(K * np + aa) * 2] = X;
                c->xn[(K * np + aa) * 2 + 1] = Y;
                double r = sqrt(X * X + Y * Y), w;
                if (r <= c->cfg.r_blend0) w = 1.0;
                else if (r >= c->cfg.r_blend1) w = 0.0;
                else { double z = (r - c->cfg.r_blend0) / (c->cfg.r_blend1 - c->cfg.r_blend0); w = 1.0 - 3.0 * z * z + 2.0 * z * z * z; }
                c->wbl[K * np + aa] = w;
                ++aa;
            }
    }
    (void)p;
}

/* ------------------------------------------------------------------ */
/* kinematics and mesh motion (Sec. 4.1 eq. defmap; blended per the     */
/* stated reading: rigid for r <= 2, cubic blend to rest at r = 8)      */
/* ------------------------------------------------------------------ */
typedef struct { const cplx *xn, *vg, *gb; } Stage;

static void motion_nodes(const pao_ctx* c, const cplx mu[3], double t, cplx* xn, cplx* vg)
{
    double w = 2.0 * M_PI / c->cfg.T;
    cplx h = mu[0] * sin(w * t), hd = mu[0] * w * cos(w * t);
    cplx th = mu[1] * csin(w * t + mu[2]), thd = mu[1] * w * ccos(w * t + mu[2]);
    cplx cs = ccos(th), sn = csin(th);
    int64_t nn = (int64_t)c->Ne * c->np;
    for (int64_t k = 0; k < nn; ++k) {
        double X = c->xn[2 * k], Y = c->xn[2 * k + 1], wb = c->wbl[k];
        /* Q = [[cos, sin], [-sin, cos]], Q' = dQ/dtheta */
        cplx qx = cs * X + sn * Y, qy = -sn * X + cs * Y;
        xn[2 * k] = X + wb * (qx - X);
        xn[2 * k + 1] = Y + wb * (qy + h - Y);
        cplx dqx = -sn * X + cs * Y, dqy = -cs * X - sn * Y;
        vg[2 * k] = wb * thd * dqx;
        vg[2 * k + 1] = wb * (thd * dqy + hd);
    }
}

/* isoparametric geometry at a reference point of element K:
 * G[i][j] = d x_i / d X_j, v_G, and the basis gradients in X */
static void point_geom(const pao_ctx* c, const Stage* S, int K, const double* phi, const double* dphi,
                       cplx G[2][2], cplx vG[2], double* dX /* [np][2] out */)
{
    int np = c->np;
    const double* jt = c->jit + 4 * K;
    G[0][0] = G[0][1] = G[1][0] = G[1][1] = 0;
    vG[0] = vG[1] = 0;
    for (int a = 0; a < np; ++a) {
        double gx = jt[0] * dphi[2 * a] + jt[1] * dphi[2 * a + 1];
        double gy = jt[2] * dphi[2 * a] + jt[3] * dphi[2 * a + 1];
        dX[2 * a] = gx; dX[2 * a + 1] = gy;
        const cplx* x = S->xn + (K * np + a) * 2;
        const cplx* v = S->vg + (K * np + a) * 2;
        G[0][0] += x[0] * gx; G[0][1] += x[0] * gy;
        G[1][0] += x[1] * gx; G[1][1] += x[1] * gy;
        vG[0] += phi[a] * v[0]; vG[1] += phi[a] * v[1];
    }
}

/* cof G = g G^{-T} and G^{-1} */
static void cof_inv(cplx G[2][2], cplx cof[2][2], cplx Gi[2][2], cplx* g)
{
    cplx det = G[0][0] * G[1][1] - G[0][1] * G[1][0];
    *g = det;
    cof[0][0] = G[1][1]; cof[0][1] = -G[1][0];
    cof[1][0] = -G[0][1]; cof[1][1] = G[0][0];
    Gi[0][0] = G[1][1] / det; Gi[0][1] = -G[0][1] / det;
    Gi[1][0] = -G[1][0] / det; Gi[1][1] = G[0][0] / det;
}

/* edge of element K across local face f: length and outward unit normal in X */
static void edge_geom(const pao_ctx* c, int K, int f, double* len, double N[2])
{
    const double* v0 = c->vxy + 2 * c->ev[3 * K + f];
    const double* v1 = c->vxy + 2 * c->ev[3 * K + (f + 1) % 3];
    double tx = v1[0] - v0[0], ty = v1[1] - v0[1];
    *len = sqrt(tx * tx + ty * ty);
    N[0] = ty / *len;
    N[1] = -tx / *len;
}

/* ------------------------------------------------------------------ */
/* GCL field gbar (reading of the GCL modification delegated in Sec. 4):  */
/*   M dgbar/dt = r_g(t),  r_g,a = -int grad phi_a . (cof G^T v_G)       */
/*                                 + oint phi_a v_G . (cof G N)           */
/* integrated with the same DIRK; gbar(0) = L2 projection of det G(0).   */
/* ------------------------------------------------------------------ */
static void gcl_rhs_all(const pao_ctx* c, const Stage* S, cplx* rg)
{
    int np = c->np, nq = c->nq, nf = c->nf;
#pragma omp parallel for schedule(static)
    for (int K = 0; K < c->Ne; ++K) {
        double dX[64];
        cplx* out = rg + (int64_t)K * np;
        for (int a = 0; a < np; ++a) out[a] = 0;
        for (int q = 0; q < nq; ++q) {
            cplx G[2][2], vG[2], cof[2][2], Gi[2][2], g;
            point_geom(c, S, K, c->phq + q * np, c->dphq + q * np * 2, G, vG, dX);
            cof_inv(G, cof, Gi, &g);
            cplx w0 = cof[0][0] * vG[0] + cof[1][0] * vG[1];
            cplx w1 = cof[0][1] * vG[0] + cof[1][1] * vG[1];
            double wq = 2.0 * c->area[K] * c->wq[q];
            for (int a = 0; a < np; ++a) out[a] -= wq * (dX[2 * a] * w0 + dX[2 * a + 1] * w1);
        }
        for (int f = 0; f < 3; ++f) {
            int nb = c->enb[3 * K + f];
            int L = K, fL = f;
            if (nb >= 0 && nb < K) { L = nb; fL = c->etw[3 * K + f]; }
            double len, N[2];
            edge_geom(c, L, fL, &len, N);
            double sgn = (L == K) ? 1.0 : -1.0;
            for (int j = 0; j < nf; ++j) {
                cplx G[2][2], vG[2], cof[2][2], Gi[2][2], g;
                point_geom(c, S, L, c->phf + (fL * nf + j) * np, c->dphf + (fL * nf + j) * np * 2, G, vG, dX);
                cof_inv(G, cof, Gi, &g);
                cplx cn0 = cof[0][0] * N[0] + cof[0][1] * N[1];
                cplx cn1 = cof[1][0] * N[0] + cof[1][1] * N[1];
                cplx flux = sgn * (vG[0] * cn0 + vG[1] * cn1);
                const double* phK = (L == K) ? c->phf + (f * nf + j) * np : c->phfr + (f * nf + j) * np;
                for (int a = 0; a < np; ++a) out[a] += len * c->wf[j] * phK[a] * flux;
            }
        }
    }
}

static double stage_time(const pao_ctx* c, int n, int i)
{
    if (n == 0) return 0.0;
    return (n - 1 + c->cc[i - 1]) * c->dt;
}
static int stage_index(int n, int i) { return n == 0 ? 0 : 1 + (n - 1) * 3 + (i - 1); }

/* gbar at every stage for parameter mu (complex for complex-step) */
static void gbar_compute(pao_ctx* c, const cplx mu[3], cplx* gb)
{
    int np = c->np, Ne = c->Ne;
    int64_t nn = (int64_t)Ne * np;
    cplx *xn = malloc(sizeof(cplx) * nn * 2), *vg = malloc(sizeof(cplx) * nn * 2);
    cplx* rg = malloc(sizeof(cplx) * nn);
    cplx* kg = malloc(sizeof(cplx) * nn * 3);
    Stage S = { xn, vg, NULL };
    /* gbar(0): L2 projection of g = det G at t = 0 */
    motion_nodes(c, mu, 0.0, xn, vg);
    for (int K = 0; K < Ne; ++K) {
        double dX[64];
        cplx proj[16];
        for (int a = 0; a < np; ++a) proj[a] = 0;
        for (int q = 0; q < c->nq; ++q) {
            cplx G[2][2], vG[2], cof[2][2], Gi[2][2], g;
            point_geom(c, &S, K, c->phq + q * np, c->dphq + q * np * 2, G, vG, dX);
            cof_inv(G, cof, Gi, &g);
            for (int a = 0; a < np; ++a) proj[a] += c->wq[q] * c->phq[q * np + a] * g;
        }
        for (int a = 0; a < np; ++a) {
            cplx s = 0;
            for (int bb = 0; bb < np; ++bb) s += c->mhi[a * np + bb] * proj[bb];
            gb[(int64_t)K * np + a] = s;
        }
    }
    cplx* prev = gb;   /* gbar^(n-1) */
    for (int n = 1; n <= c->Nt; ++n) {
        for (int i = 1; i <= 3; ++i) {
            motion_nodes(c, mu, stage_time(c, n, i), xn, vg);
            gcl_rhs_all(c, &S, rg);
            /* kg_i = dt M^{-1} r_g */
            for (int K = 0; K < Ne; ++K)
                for (int a = 0; a < np; ++a) {
                    cplx s = 0;
                    for (int bb = 0; bb < np; ++bb) s += c->mhi[a * np + bb] * rg[(int64_t)K * np + bb];
                    kg[(int64_t)(i - 1) * nn + (int64_t)K * np + a] = c->dt * s / (2.0 * c->area[K]);
                }
            cplx* cur = gb + (int64_t)stage_index(n, i) * nn;
            for (int64_t k = 0; k < nn; ++k) {
                cplx s = prev[k];
                for (int j = 1; j <= i; ++j) s += c->A[i - 1][j - 1] * kg[(int64_t)(j - 1) * nn + k];
                cur[k] = s;
            }
        }
        /* stiffly accurate tableau: gbar^(n) = last stage value */
        prev = gb + (int64_t)stage_index(n, 3) * nn;
    }
    free(xn); free(vg); free(rg); free(kg);
}

/* ------------------------------------------------------------------ */
/* physics: compressible Navier-Stokes (Sec. 4, eqs. ns1-ns5), 2-D       */
/* ------------------------------------------------------------------ */
static void flux_inv(const pao_ctx* c, const cplx U[4], cplx F[4][2])
{
    cplx r = U[0], ux = U[1] / r, uy = U[2] / r;
    cplx p = (c->gam - 1.0) * (U[3] - 0.5 * r * (ux * ux + uy * uy));
    F[0][0] = U[1];          F[0][1] = U[2];
    F[1][0] = U[1] * ux + p; F[1][1] = U[1] * uy;
    F[2][0] = U[2] * ux;     F[2][1] = U[2] * uy + p;
    F[3][0] = (U[3] + p) * ux; F[3][1] = (U[3] + p) * uy;
}

/* viscous flux from the state and its physical gradient dU[m][d];
 * heat = 0 drops the heat flux (adiabatic wall) */
static void flux_vis(const pao_ctx* c, const cplx U[4], cplx dU[4][2], cplx F[4][2], int heat)
{
    cplx r = U[0], u[2] = { U[1] / r, U[2] / r }, E = U[3] / r;
    cplx du[2][2], dE[2];
    for (int d = 0; d < 2; ++d) {
        du[0][d] = (dU[1][d] - u[0] * dU[0][d]) / r;
        du[1][d] = (dU[2][d] - u[1] * dU[0][d]) / r;
        dE[d] = (dU[3][d] - E * dU[0][d]) / r;
    }
    cplx div = du[0][0] + du[1][1];
    cplx tau[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) tau[i][j] = c->muv * (du[i][j] + du[j][i] - (i == j ? 2.0 / 3.0 * div : 0.0));
    for (int d = 0; d < 2; ++d) {
        /* h = E + p/rho - |u|^2/2 = gamma (E - |u|^2/2);  q = -(mu/Pr) grad h */
        cplx dh = c->gam * (dE[d] - u[0] * du[0][d] - u[1] * du[1][d]);
        cplx q = heat ? -(c->muv / c->pr) * dh : 0.0;
        F[0][d] = 0;
        F[1][d] = tau[0][d];
        F[2][d] = tau[1][d];
        F[3][d] = u[0] * tau[0][d] + u[1] * tau[1][d] - q;
    }
}

/* H(U) = F_inv(U) n - U (v_G . n) */
static void flux_H(const pao_ctx* c, const cplx U[4], const cplx n[2], cplx vn, cplx H[4])
{
    cplx F[4][2];
    flux_inv(c, U, F);
    for (int m = 0; m < 4; ++m) H[m] = F[m][0] * n[0] + F[m][1] * n[1] - U[m] * vn;
}

/* smoothed local Lax-Friedrichs flux (reading; the paper names no Riemann
 * solver): Fhat = (H- + H+)/2 - alpha (U+ - U-)/2, alpha = (s- + s+)/2,
 * s = sqrt((u.n - v_G.n)^2 + delta^2) + c */
static void flux_lf(const pao_ctx* c, const cplx UL[4], const cplx UR[4], const cplx n[2], cplx vn, cplx Fh[4])
{
    cplx HL[4], HR[4];
    flux_H(c, UL, n, vn, HL);
    flux_H(c, UR, n, vn, HR);
    cplx s[2];
    const cplx* Us[2] = { UL, UR };
    for (int k = 0; k < 2; ++k) {
        const cplx* U = Us[k];
        cplx r = U[0], ux = U[1] / r, uy = U[2] / r;
        cplx p = (c->gam - 1.0) * (U[3] - 0.5 * r * (ux * ux + uy * uy));
        cplx un = ux * n[0] + uy * n[1] - vn;
        s[k] = csqrt(un * un + LF_DELTA * LF_DELTA) + csqrt(c->gam * p / r);
    }
    cplx al = 0.5 * (s[0] + s[1]);
    for (int m = 0; m < 4; ++m) Fh[m] = 0.5 * (HL[m] + HR[m]) - 0.5 * al * (UR[m] - UL[m]);
}

/* physical state U = U_X / gbar and its X-gradient at a point of element K */
static void point_state(const pao_ctx* c, const Stage* S, int K, const cplx* u, const double* phi,
                        const double* dX, cplx U[4], cplx gU[4][2])
{
    int np = c->np;
    cplx UX[4] = { 0, 0, 0, 0 }, dUX[4][2] = { { 0 } }, g = 0, dg[2] = { 0, 0 };
    for (int a = 0; a < np; ++a) {
        const cplx* ua = u + ((int64_t)K * np + a) * 4;
        cplx ga = S->gb[(int64_t)K * np + a];
        g += phi[a] * ga;
        dg[0] += dX[2 * a] * ga;
        dg[1] += dX[2 * a + 1] * ga;
        for (int m = 0; m < 4; ++m) {
            UX[m] += phi[a] * ua[m];
            dUX[m][0] += dX[2 * a] * ua[m];
            dUX[m][1] += dX[2 * a + 1] * ua[m];
        }
    }
    for (int m = 0; m < 4; ++m) {
        U[m] = UX[m] / g;
        if (gU) {
            gU[m][0] = (dUX[m][0] - U[m] * dg[0]) / g;
            gU[m][1] = (dUX[m][1] - U[m] * dg[1]) / g;
        }
    }
}

/* basis gradients in X for element K from reference gradients */
static void grad_X(const pao_ctx* c, int K, const double* dphi, double* dX)
{
    const double* jt = c->jit + 4 * K;
    for (int a = 0; a < c->np; ++a) {
        dX[2 * a] = jt[0] * dphi[2 * a] + jt[1] * dphi[2 * a + 1];
        dX[2 * a + 1] = jt[2] * dphi[2 * a] + jt[3] * dphi[2 * a + 1];
    }
}

/* Interior face between L < R (local faces fL, fR), in L's orientation.
 * Viscous treatment (reading of the compact DG method cited in Sec. 4):
 *   trace  Uhat = U^R;  lifting r_e on L:
 *     int_L r_e : tau = - int_e (U^L - U^R) (x) N^L : tau
 *   face viscous flux  F_vis(U^L, grad_X U^L + r_e) (one-sided, C11 = 0).
 * Outputs the flux Fhat . N^L at the nf points and the lifting coefficients
 * lift[c][m][D] (nodal, on L). */
static void face_interior(const pao_ctx* c, const Stage* S, int L, int fL, int R, int fR, const cplx* u,
                          cplx* Fh /* [nf][4] */, cplx* lift /* [np][4][2] */)
{
    int np = c->np, nf = c->nf;
    double len, N[2];
    edge_geom(c, L, fL, &len, N);
    cplx UL[8][4], UR[8][4], gUL[8][4][2];
    double dXL[64], dXR[64];
    for (int j = 0; j < nf; ++j) {
        const double* phL = c->phf + (fL * nf + j) * np;
        const double* phR = c->phfr + (fR * nf + j) * np;
        grad_X(c, L, c->dphf + (fL * nf + j) * np * 2, dXL);
        grad_X(c, R, c->dphfr + (fR * nf + j) * np * 2, dXR);
        point_state(c, S, L, u, phL, dXL, UL[j], gUL[j]);
        point_state(c, S, R, u, phR, dXR, UR[j], NULL);
    }
    double s = -len / (2.0 * c->area[L]);
    for (int cc = 0; cc < np; ++cc)
        for (int m = 0; m < 4; ++m) {
            cplx acc = 0;
            for (int cp = 0; cp < np; ++cp) {
                cplx t = 0;
                for (int j = 0; j < nf; ++j) t += c->wf[j] * c->phf[(fL * nf + j) * np + cp] * (UL[j][m] - UR[j][m]);
                acc += c->mhi[cc * np + cp] * t;
            }
            lift[(cc * 4 + m) * 2] = s * acc * N[0];
            lift[(cc * 4 + m) * 2 + 1] = s * acc * N[1];
        }
    for (int j = 0; j < nf; ++j) {
        const double* phL = c->phf + (fL * nf + j) * np;
        cplx G[2][2], vG[2], cof[2][2], Gi[2][2], g;
        point_geom(c, S, L, phL, c->dphf + (fL * nf + j) * np * 2, G, vG, dXL);
        cof_inv(G, cof, Gi, &g);
        cplx cn[2] = { cof[0][0] * N[0] + cof[0][1] * N[1], cof[1][0] * N[0] + cof[1][1] * N[1] };
        cplx jf = csqrt(cn[0] * cn[0] + cn[1] * cn[1]);
        cplx nn[2] = { cn[0] / jf, cn[1] / jf };
        cplx vn = vG[0] * nn[0] + vG[1] * nn[1];
        cplx Fi[4];
        flux_lf(c, UL[j], UR[j], nn, vn, Fi);
        cplx q[4][2], dU[4][2], Fv[4][2];
        for (int m = 0; m < 4; ++m)
            for (int D = 0; D < 2; ++D) {
                cplx t = gUL[j][m][D];
                for (int cc = 0; cc < np; ++cc) t += phL[cc] * lift[(cc * 4 + m) * 2 + D];
                q[m][D] = t;
            }
        for (int m = 0; m < 4; ++m)
            for (int d = 0; d < 2; ++d) dU[m][d] = q[m][0] * Gi[0][d] + q[m][1] * Gi[1][d];
        flux_vis(c, UL[j], dU, Fv, 1);
        for (int m = 0; m < 4; ++m) Fh[j * 4 + m] = jf * Fi[m] - (Fv[m][0] * cn[0] + Fv[m][1] * cn[1]);
    }
}

/* Boundary face of K.  Far field (reading of the characteristic free-stream
 * condition): Lax-Friedrichs flux against U_inf plus the interior viscous
 * flux.  Wall (no-slip, adiabatic; reading): the Lax-Friedrichs flux
 * against the reflected state U_b (interior density and pressure, velocity
 * 2 v_G - u, so that the mass flux vanishes and the average velocity is the
 * wall's), interior viscous stress with zero heat flux, and an
 * interior-penalty term mu C11 rho (u - v_G) on the momentum with
 * C11 = 10 / h, h = 2|K| / |e|.  Fh [nf][4] is Fhat . N_K. */
static void face_boundary(const pao_ctx* c, const Stage* S, int K, int f, int wall, const cplx* u, cplx* Fh)
{
    int np = c->np, nf = c->nf;
    double len, N[2], dX[64];
    edge_geom(c, K, f, &len, N);
    for (int j = 0; j < nf; ++j) {
        const double* ph = c->phf + (f * nf + j) * np;
        cplx G[2][2], vG[2], cof[2][2], Gi[2][2], g;
        point_geom(c, S, K, ph, c->dphf + (f * nf + j) * np * 2, G, vG, dX);
        cof_inv(G, cof, Gi, &g);
        cplx U[4], gU[4][2], dU[4][2];
        point_state(c, S, K, u, ph, dX, U, gU);
        for (int m = 0; m < 4; ++m)
            for (int d = 0; d < 2; ++d) dU[m][d] = gU[m][0] * Gi[0][d] + gU[m][1] * Gi[1][d];
        cplx cn[2] = { cof[0][0] * N[0] + cof[0][1] * N[1], cof[1][0] * N[0] + cof[1][1] * N[1] };
        cplx jf = csqrt(cn[0] * cn[0] + cn[1] * cn[1]);
        cplx nn[2] = { cn[0] / jf, cn[1] / jf };
        cplx vn = vG[0] * nn[0] + vG[1] * nn[1];
        if (!wall) {
            cplx Ui[4] = { c->Uinf[0], c->Uinf[1], c->Uinf[2], c->Uinf[3] };
            cplx Fi[4], Fv[4][2];
            flux_lf(c, U, Ui, nn, vn, Fi);
            flux_vis(c, U, dU, Fv, 1);
            for (int m = 0; m < 4; ++m) Fh[j * 4 + m] = jf * Fi[m] - (Fv[m][0] * cn[0] + Fv[m][1] * cn[1]);
        } else {
            cplx r = U[0], ux = U[1] / r, uy = U[2] / r;
            /* reflected state: interior density and pressure, velocity 2 v_G - u */
            cplx bx = 2.0 * vG[0] - ux, by = 2.0 * vG[1] - uy;
            cplx Ub[4] = { r, r * bx, r * by, U[3] - 0.5 * r * (ux * ux + uy * uy) + 0.5 * r * (bx * bx + by * by) };
            cplx H[4], Fv[4][2];
            flux_lf(c, U, Ub, nn, vn, H);
            flux_vis(c, U, dU, Fv, 0);
            cplx tn0 = Fv[1][0] * nn[0] + Fv[1][1] * nn[1];
            cplx tn1 = Fv[2][0] * nn[0] + Fv[2][1] * nn[1];
            double C11 = WALL_ETA / (2.0 * c->area[K] / len);
            Fh[j * 4 + 0] = jf * H[0];
            Fh[j * 4 + 1] = jf * (H[1] - tn0 + c->muv * C11 * r * (ux - vG[0]));
            Fh[j * 4 + 2] = jf * (H[2] - tn1 + c->muv * C11 * r * (uy - vG[1]));
            Fh[j * 4 + 3] = jf * (H[3] - (vG[0] * tn0 + vG[1] * tn1));
        }
    }
}

/* Residual rows of element K (DG weak form on the fixed reference mesh):
 *   r_{K,a} = int_K grad_X phi_a . F_X dX - oint_{dK} phi_a Fhat . N dS
 *   F_X = [F_inv(U) - F_vis(U, q G^{-1})] cof G - U (x) (cof G^T v_G),
 *   q = grad_X U + sum of liftings of the faces where K is the L side. */
static void elem_residual(const pao_ctx* c, const Stage* S, int K, const cplx* u, cplx* out)
{
    int np = c->np, nf = c->nf, b = c->b;
    cplx Fh[8 * 4], lift[3][16 * 8];
    int has[3] = { 0, 0, 0 };
    for (int k = 0; k < b; ++k) out[k] = 0;
    for (int f = 0; f < 3; ++f) {
        int nb = c->enb[3 * K + f];
        double len, N[2];
        edge_geom(c, K, f, &len, N);
        if (nb >= 0) {
            int tw = c->etw[3 * K + f];
            int L, fL, R, fR;
            if (K < nb) { L = K; fL = f; R = nb; fR = tw; }
            else { L = nb; fL = tw; R = K; fR = f; }
            cplx lf[16 * 8];
            face_interior(c, S, L, fL, R, fR, u, Fh, lf);
            double sgn = (K == L) ? 1.0 : -1.0;
            const double* phK = (K == L) ? c->phf + f * nf * np : c->phfr + f * nf * np;
            for (int j = 0; j < nf; ++j)
                for (int a = 0; a < np; ++a)
                    for (int m = 0; m < 4; ++m) out[a * 4 + m] -= sgn * len * c->wf[j] * phK[j * np + a] * Fh[j * 4 + m];
            if (K == L) { memcpy(lift[f], lf, sizeof(cplx) * np * 8); has[f] = 1; }
        } else {
            int wall = (nb == -1) && !c->cfg.wall_is_farfield;
            face_boundary(c, S, K, f, wall, u, Fh);
            const double* phK = c->phf + f * nf * np;
            for (int j = 0; j < nf; ++j)
                for (int a = 0; a < np; ++a)
                    for (int m = 0; m < 4; ++m) out[a * 4 + m] -= len * c->wf[j] * phK[j * np + a] * Fh[j * 4 + m];
        }
    }
    double dX[64];
    for (int q = 0; q < c->nq; ++q) {
        const double* ph = c->phq + q * np;
        cplx G[2][2], vG[2], cof[2][2], Gi[2][2], g;
        point_geom(c, S, K, ph, c->dphq + q * np * 2, G, vG, dX);
        cof_inv(G, cof, Gi, &g);
        cplx U[4], gU[4][2], dU[4][2], Fi[4][2], Fv[4][2];
        point_state(c, S, K, u, ph, dX, U, gU);
        for (int f = 0; f < 3; ++f)
            if (has[f])
                for (int m = 0; m < 4; ++m)
                    for (int D = 0; D < 2; ++D)
                        for (int cc = 0; cc < np; ++cc) gU[m][D] += ph[cc] * lift[f][(cc * 4 + m) * 2 + D];
        for (int m = 0; m < 4; ++m)
            for (int d = 0; d < 2; ++d) dU[m][d] = gU[m][0] * Gi[0][d] + gU[m][1] * Gi[1][d];
        flux_inv(c, U, Fi);
        flux_vis(c, U, dU, Fv, 1);
        cplx w0 = cof[0][0] * vG[0] + cof[1][0] * vG[1];
        cplx w1 = cof[0][1] * vG[0] + cof[1][1] * vG[1];
        double wq = 2.0 * c->area[K] * c->wq[q];
        for (int m = 0; m < 4; ++m) {
            cplx FX0 = (Fi[m][0] - Fv[m][0]) * cof[0][0] + (Fi[m][1] - Fv[m][1]) * cof[1][0] - U[m] * w0;
            cplx FX1 = (Fi[m][0] - Fv[m][0]) * cof[0][1] + (Fi[m][1] - Fv[m][1]) * cof[1][1] - U[m] * w1;
            for (int a = 0; a < np; ++a) out[a * 4 + m] += wq * (dX[2 * a] * FX0 + dX[2 * a + 1] * FX1);
        }
    }
}

/* instantaneous QoI contributions of element K's wall faces (Sec. 4 eq. qoi,
 * solver-consistent reading): the force on the body is the momentum part of
 * the wall numerical flux integrated over the wall; P = f . v_G, F_x = f . e1 */
static void elem_qoi(const pao_ctx* c, const Stage* S, int K, const cplx* u, cplx f[2])
{
    int np = c->np, nf = c->nf;
    f[0] = f[1] = 0;
    if (c->cfg.wall_is_farfield) return;
    for (int fc = 0; fc < 3; ++fc) {
        if (c->enb[3 * K + fc] != -1) continue;
        double len, N[2], dX[64];
        edge_geom(c, K, fc, &len, N);
        cplx Fh[8 * 4];
        face_boundary(c, S, K, fc, 1, u, Fh);
        for (int j = 0; j < nf; ++j) {
            cplx G[2][2], vG[2];
            point_geom(c, S, K, c->phf + (fc * nf + j) * np, c->dphf + (fc * nf + j) * np * 2, G, vG, dX);
            cplx w = len * c->wf[j];
            f[0] += w * (Fh[j * 4 + 1] * vG[0] + Fh[j * 4 + 2] * vG[1]);
            f[1] += w * Fh[j * 4 + 1];
        }
    }
}

/* ------------------------------------------------------------------ */
/* stage data, residual, Jacobian, derivatives in mu                    */
/* ------------------------------------------------------------------ */
typedef struct { cplx *xn, *vg; } Motion;

static void motion_alloc(const pao_ctx* c, Motion* m)
{
    int64_t nn = (int64_t)c->Ne * c->np;
    m->xn = malloc(sizeof(cplx) * nn * 2);
    m->vg = malloc(sizeof(cplx) * nn * 2);
}
static void motion_free(Motion* m) { free(m->xn); free(m->vg); }

/* stage data for stage (n, i); dir = 0 real parameters, dir = 1..3 complex
 * step in mu_{dir-1} */
static Stage stage_make(pao_ctx* c, int n, int i, int dir, Motion* m)
{
    cplx mu[3] = { c->mu[0], c->mu[1], c->mu[2] };
    if (dir > 0) mu[dir - 1] += I * CSTEP;
    motion_nodes(c, mu, stage_time(c, n, i), m->xn, m->vg);
    int64_t nn = (int64_t)c->Ne * c->np;
    Stage S = { m->xn, m->vg, c->gb[dir] + (int64_t)stage_index(n, i) * nn };
    return S;
}

static int check_stage(pao_ctx* c, int n, int i)
{
    if (!c->have_params) return fail(c, -4, "parameters not set");
    if (!((n == 0 && i == 0) || (n >= 1 && n <= c->Nt && i >= 1 && i <= 3)))
        return fail(c, -1, "bad stage (%d, %d)", n, i);
    return 0;
}

static int ensure_dgb(pao_ctx* c)
{
    if (c->have_dgb) return 0;
    int64_t nn = (int64_t)c->Ne * c->np * (c->nst + 1);
    for (int k = 1; k <= 3; ++k) {
        if (!c->gb[k]) c->gb[k] = malloc(sizeof(cplx) * nn);
        cplx mu[3] = { c->mu[0], c->mu[1], c->mu[2] };
        mu[k - 1] += I * CSTEP;
        gbar_compute(c, mu, c->gb[k]);
    }
    c->have_dgb = 1;
    return 0;
}

static void residual_stage(pao_ctx* c, const Stage* S, const cplx* uc, double* r, double* rim)
{
    int b = c->b;
#pragma omp parallel for schedule(static)
    for (int K = 0; K < c->Ne; ++K) {
        cplx out[64 * 4];
        elem_residual(c, S, K, uc, out);
        for (int k = 0; k < b; ++k) {
            if (r) r[(int64_t)K * b + k] = creal(out[k]);
            if (rim) rim[(int64_t)K * b + k] = cimag(out[k]) / CSTEP;
        }
    }
}

static cplx* to_cplx(const pao_ctx* c, const double* u)
{
    cplx* uc = malloc(sizeof(cplx) * c->Nu);
    for (int64_t k = 0; k < c->Nu; ++k) uc[k] = u[k];
    return uc;
}

static void jacobian_stage(pao_ctx* c, const Stage* S, const double* u, double* blk)
{
    int b = c->b, Ne = c->Ne;
    memset(blk, 0, sizeof(double) * (size_t)Ne * 4 * b * b);
#pragma omp parallel
    {
        cplx* uc = to_cplx(c, u);
        cplx out[64 * 4];
#pragma omp for schedule(static)
        for (int Kp = 0; Kp < Ne; ++Kp) {
            for (int col = 0; col < b; ++col) {
                int64_t idx = (int64_t)Kp * b + col;
                uc[idx] = u[idx] + I * CSTEP;
                /* rows of Kp itself */
                elem_residual(c, S, Kp, uc, out);
                for (int row = 0; row < b; ++row)
                    blk[(((int64_t)Kp * 4 + 0) * b + row) * b + col] = cimag(out[row]) / CSTEP;
                /* rows of the neighbours */
                for (int f = 0; f < 3; ++f) {
                    int nb = c->enb[3 * Kp + f];
                    if (nb < 0) continue;
                    int slot = 1 + c->etw[3 * Kp + f];
                    elem_residual(c, S, nb, uc, out);
                    for (int row = 0; row < b; ++row)
                        blk[(((int64_t)nb * 4 + slot) * b + row) * b + col] = cimag(out[row]) / CSTEP;
                }
                uc[idx] = u[idx];
            }
        }
        free(uc);
    }
}

/* dr/dmu_k at a stage: complex step in mu through the mesh motion and gbar */
static void drdmu_stage(pao_ctx* c, int n, int i, const double* u, double* out)
{
    ensure_dgb(c);
    cplx* uc = to_cplx(c, u);
    Motion m;
    motion_alloc(c, &m);
    for (int k = 0; k < 3; ++k) {
        Stage S = stage_make(c, n, i, k + 1, &m);
        residual_stage(c, &S, uc, NULL, out + (int64_t)k * c->Nu);
    }
    motion_free(&m);
    free(uc);
}

/* QoIs, d/du (complex step per wall-element DOF) and d/dmu */
static void qoi_stage(pao_ctx* c, int n, int i, const double* u, double f[2], double* dfdu, double* dfdmu)
{
    Motion m;
    motion_alloc(c, &m);
    cplx* uc = to_cplx(c, u);
    Stage S = stage_make(c, n, i, 0, &m);
    double acc[2] = { 0, 0 };
    if (dfdu) memset(dfdu, 0, sizeof(double) * 2 * c->Nu);
    for (int K = 0; K < c->Ne; ++K) {
        int wall = 0;
        for (int fc = 0; fc < 3; ++fc) wall |= (c->enb[3 * K + fc] == -1);
        if (!wall) continue;
        cplx fk[2];
        elem_qoi(c, &S, K, uc, fk);
        acc[0] += creal(fk[0]);
        acc[1] += creal(fk[1]);
        if (dfdu)
            for (int col = 0; col < c->b; ++col) {
                int64_t idx = (int64_t)K * c->b + col;
                uc[idx] = u[idx] + I * CSTEP;
                elem_qoi(c, &S, K, uc, fk);
                dfdu[idx] = cimag(fk[0]) / CSTEP;
                dfdu[c->Nu + idx] = cimag(fk[1]) / CSTEP;
                uc[idx] = u[idx];
            }
    }
    if (f) { f[0] = acc[0]; f[1] = acc[1]; }
    if (dfdmu) {
        ensure_dgb(c);
        for (int k = 0; k < 3; ++k) {
            Stage Sk = stage_make(c, n, i, k + 1, &m);
            double d0 = 0, d1 = 0;
            for (int K = 0; K < c->Ne; ++K) {
                cplx fk[2];
                elem_qoi(c, &Sk, K, uc, fk);
                d0 += cimag(fk[0]) / CSTEP;
                d1 += cimag(fk[1]) / CSTEP;
            }
            dfdmu[k] = d0;       /* P  */
            dfdmu[3 + k] = d1;   /* F_x */
        }
    }
    free(uc);
    motion_free(&m);
}

/* ------------------------------------------------------------------ */
/* linear algebra on the block-sparse operators                         */
/* ------------------------------------------------------------------ */
void pao_mass_apply(const pao_ctx* c, const double* x, double* y)
{
    int np = c->np;
    for (int K = 0; K < c->Ne; ++K) {
        double s2 = 2.0 * c->area[K];
        for (int a = 0; a < np; ++a)
            for (int m = 0; m < 4; ++m) {
                double s = 0;
                for (int bb = 0; bb < np; ++bb) s += c->mh[a * np + bb] * x[((int64_t)K * np + bb) * 4 + m];
                y[((int64_t)K * np + a) * 4 + m] = s2 * s;
            }
    }
}

void pao_bsr_apply(const pao_ctx* c, const double* blk, int32_t tr, const double* x, double* y)
{
    int b = c->b;
    memset(y, 0, sizeof(double) * c->Nu);
    for (int K = 0; K < c->Ne; ++K)
        for (int s = 0; s < 4; ++s) {
            int col = s == 0 ? K : c->enb[3 * K + s - 1];
            if (col < 0) continue;
            const double* B = blk + ((int64_t)K * 4 + s) * b * b;
            if (!tr) {
                for (int i = 0; i < b; ++i) {
                    double acc = 0;
                    for (int j = 0; j < b; ++j) acc += B[i * b + j] * x[(int64_t)col * b + j];
                    y[(int64_t)K * b + i] += acc;
                }
            } else {
                for (int j = 0; j < b; ++j) {
                    double acc = 0;
                    for (int i = 0; i < b; ++i) acc += B[i * b + j] * x[(int64_t)K * b + i];
                    y[(int64_t)col * b + j] += acc;
                }
            }
        }
}

/* stage operator A = M - a_dt J (or its transpose) */
typedef struct {
    pao_ctx* c;
    const double* J;
    double adt;
    int tr;
    double* tmp;
    double* dlu;   /* LU of diagonal blocks of A */
    int* dpiv;
} StageOp;

static void stageop_apply(void* ctx, const double* x, double* y)
{
    StageOp* o = ctx;
    pao_mass_apply(o->c, x, y);
    pao_bsr_apply(o->c, o->J, o->tr, x, o->tmp);
    for (int64_t k = 0; k < o->c->Nu; ++k) y[k] -= o->adt * o->tmp[k];
}

static void stageop_prec(void* ctx, const double* x, double* z)
{
    StageOp* o = ctx;
    int b = o->c->b;
    memcpy(z, x, sizeof(double) * o->c->Nu);
    for (int K = 0; K < o->c->Ne; ++K)
        lu_solve(b, o->dlu + (int64_t)K * b * b, o->dpiv + (int64_t)K * b, z + (int64_t)K * b, o->tr);
}

typedef void (*apply_fn)(void*, const double*, double*);

/* GMRES with right preconditioning (prec may be NULL), zero initial guess,
 * modified Gram-Schmidt Arnoldi and Givens rotations; stops when the residual
 * norm estimate is <= rtol ||b||.  Returns the number of iterations or -2. */
static int gmres(int64_t n, apply_fn A, apply_fn P, void* ctx, const double* bvec, double* x,
                 double rtol, int restart, int maxit, double* relres)
{
    double bn = nrm2(n, bvec);
    memset(x, 0, sizeof(double) * n);
    if (relres) *relres = 0;
    if (bn == 0.0) return 0;
    int m = restart;
    double* V = malloc(sizeof(double) * n * (m + 1));
    double* H = calloc((size_t)(m + 1) * m, sizeof(double));
    double *cs = malloc(sizeof(double) * m), *sn = malloc(sizeof(double) * m), *g = malloc(sizeof(double) * (m + 1));
    double *w = malloc(sizeof(double) * n), *z = malloc(sizeof(double) * n), *y = malloc(sizeof(double) * m);
    int total = 0, conv = 0;
    double res = bn;
    while (total < maxit) {
        /* r = b - A x */
        A(ctx, x, w);
        for (int64_t k = 0; k < n; ++k) w[k] = bvec[k] - w[k];
        double beta = nrm2(n, w);
        res = beta;
        if (beta <= rtol * bn) { conv = 1; break; }
        for (int64_t k = 0; k < n; ++k) V[k] = w[k] / beta;
        memset(g, 0, sizeof(double) * (m + 1));
        g[0] = beta;
        int j = 0;
        for (; j < m && total < maxit; ++j) {
            ++total;
            double* vj = V + (int64_t)j * n;
            if (P) { P(ctx, vj, z); A(ctx, z, w); } else A(ctx, vj, w);
            for (int i = 0; i <= j; ++i) {
                double h = dot(n, w, V + (int64_t)i * n);
                H[i * m + j] = h;
                for (int64_t k = 0; k < n; ++k) w[k] -= h * V[(int64_t)i * n + k];
            }
            double hn = nrm2(n, w);
            H[(j + 1) * m + j] = hn;
            for (int i = 0; i < j; ++i) {
                double a = H[i * m + j], bb = H[(i + 1) * m + j];
                H[i * m + j] = cs[i] * a + sn[i] * bb;
                H[(i + 1) * m + j] = -sn[i] * a + cs[i] * bb;
            }
            double a = H[j * m + j], bb = H[(j + 1) * m + j];
            double rr = sqrt(a * a + bb * bb);
            cs[j] = a / rr; sn[j] = bb / rr;
            H[j * m + j] = rr; H[(j + 1) * m + j] = 0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            res = fabs(g[j + 1]);
            if (res <= rtol * bn || hn == 0.0) { ++j; break; }
            for (int64_t k = 0; k < n; ++k) V[(int64_t)(j + 1) * n + k] = w[k] / hn;
        }
        /* y = H^{-1} g, x += P^{-1} V y */
        for (int i = j - 1; i >= 0; --i) {
            double s = g[i];
            for (int k = i + 1; k < j; ++k) s -= H[i * m + k] * y[k];
            y[i] = s / H[i * m + i];
        }
        memset(w, 0, sizeof(double) * n);
        for (int i = 0; i < j; ++i)
            for (int64_t k = 0; k < n; ++k) w[k] += y[i] * V[(int64_t)i * n + k];
        if (P) { P(ctx, w, z); for (int64_t k = 0; k < n; ++k) x[k] += z[k]; }
        else for (int64_t k = 0; k < n; ++k) x[k] += w[k];
        if (res <= rtol * bn) {
            /* confirm with the true residual */
            A(ctx, x, w);
            for (int64_t k = 0; k < n; ++k) w[k] = bvec[k] - w[k];
            res = nrm2(n, w);
            if (res <= rtol * bn * 10.0) { conv = 1; break; }
        }
    }
    free(V); free(H); free(cs); free(sn); free(g); free(w); free(z); free(y);
    if (relres) *relres = res / bn;
    return conv ? total : -2;
}

int pao_stage_solve(pao_ctx* c, const double* J, double adt, int32_t tr, const double* rhs, double* x)
{
    int b = c->b, Ne = c->Ne;
    int64_t Nu = c->Nu;
    if (c->cfg.lin_solver == 0) {
        /* dense LU of the assembled operator */
        double* D = calloc((size_t)Nu * Nu, sizeof(double));
        int* piv = malloc(sizeof(int) * Nu);
        for (int K = 0; K < Ne; ++K) {
            double s2 = 2.0 * c->area[K];
            for (int a = 0; a < c->np; ++a)
                for (int bb = 0; bb < c->np; ++bb)
                    for (int m = 0; m < 4; ++m)
                        D[((int64_t)K * b + a * 4 + m) * Nu + (int64_t)K * b + bb * 4 + m] += s2 * c->mh[a * c->np + bb];
            for (int s = 0; s < 4; ++s) {
                int col = s == 0 ? K : c->enb[3 * K + s - 1];
                if (col < 0) continue;
                const double* B = J + ((int64_t)K * 4 + s) * b * b;
                for (int i = 0; i < b; ++i)
                    for (int j = 0; j < b; ++j) D[((int64_t)K * b + i) * Nu + (int64_t)col * b + j] -= adt * B[i * b + j];
            }
        }
        int rc = lu_factor((int)Nu, D, piv);
        if (rc) { free(D); free(piv); return fail(c, -3, "singular stage operator"); }
        memcpy(x, rhs, sizeof(double) * Nu);
        lu_solve((int)Nu, D, piv, x, tr);
        free(D); free(piv);
        c->cnt_lin += 1;
        return 1;
    }
    StageOp o = { c, J, adt, tr, malloc(sizeof(double) * Nu), malloc(sizeof(double) * (size_t)Ne * b * b),
                  malloc(sizeof(int) * (size_t)Ne * b) };
    for (int K = 0; K < Ne; ++K) {
        double* d = o.dlu + (int64_t)K * b * b;
        const double* B = J + ((int64_t)K * 4) * b * b;
        double s2 = 2.0 * c->area[K];
        for (int i = 0; i < b; ++i)
            for (int j = 0; j < b; ++j) {
                double mm = ((i & 3) == (j & 3)) ? s2 * c->mh[(i >> 2) * c->np + (j >> 2)] : 0.0;
                d[i * b + j] = mm - adt * B[i * b + j];
            }
        if (lu_factor(b, d, o.dpiv + (int64_t)K * b)) {
            free(o.tmp); free(o.dlu); free(o.dpiv);
            return fail(c, -3, "singular diagonal block %d", K);
        }
    }
    double rr;
    int its = gmres(Nu, stageop_apply, stageop_prec, &o, rhs, x, c->cfg.lin_rtol, c->cfg.gmres_restart,
                    100000, &rr);
    free(o.tmp); free(o.dlu); free(o.dpiv);
    if (its < 0) return fail(c, -2, "stage GMRES did not converge (rel res %.3e)", rr);
    c->cnt_lin += its;
    return its;
}

/* ------------------------------------------------------------------ */
/* DIRK3: Alexander's L-stable three-stage scheme (reading; the paper     */
/* says "third-order DIRK" only)                                        */
/* ------------------------------------------------------------------ */
void pao_dirk_tableau(double A[9], double b[3], double cc[3])
{
    /* alpha: root of x^3 - 3x^2 + 3x/2 - 1/6 in (1/6, 1/2) */
    double x = 0.44;
    for (int it = 0; it < 60; ++it) {
        double f = x * x * x - 3 * x * x + 1.5 * x - 1.0 / 6.0, d = 3 * x * x - 6 * x + 1.5;
        x -= f / d;
    }
    double al = x, t2 = 0.5 * (1.0 + al);
    double b1 = -(6 * al * al - 16 * al + 1) / 4.0, b2 = (6 * al * al - 20 * al + 5) / 4.0;
    double AA[9] = { al, 0, 0, t2 - al, al, 0, b1, b2, al };
    memcpy(A, AA, sizeof AA);
    b[0] = b1; b[1] = b2; b[2] = al;
    cc[0] = al; cc[1] = t2; cc[2] = 1.0;
}

/* ------------------------------------------------------------------ */
/* public API                                                           */
/* ------------------------------------------------------------------ */
void pao_default_config(pao_config* c)
{
    memset(c, 0, sizeof *c);
    c->Nr = 8; c->Nth = 24; c->p = 1; c->Nt = 20;
    c->r_far = 10.0; c->stretch = 1.3;
    c->mach = 0.2; c->re = 1000.0; c->gamma = 1.4; c->pr = 0.72;
    c->T = 1.0; c->r_blend0 = 2.0; c->r_blend1 = 8.0;
    c->wall_is_farfield = 0;
    c->lin_solver = 1; c->gmres_restart = 30; c->lin_rtol = 1e-12;
    c->newton_atol = 1e-11; c->newton_maxit = 20; c->nthreads = 0;
}

pao_ctx* pao_create(const pao_config* cfg)
{
    if (!cfg || cfg->Nr < 1 || cfg->Nth < 3 || cfg->p < 1 || cfg->p > 4 || cfg->Nt < 1) return NULL;
    pao_ctx* c = calloc(1, sizeof *c);
    c->cfg = *cfg;
#ifdef _OPENMP
    if (cfg->nthreads > 0) omp_set_num_threads(cfg->nthreads);
#endif
    if (ref_init(c)) { free(c); return NULL; }
    mesh_init(c);
    c->Nu = (int64_t)c->Ne * c->b;
    c->Nt = cfg->Nt;
    c->nst = 3 * cfg->Nt;
    c->gam = cfg->gamma;
    c->muv = 1.0 / cfg->re;
    c->pr = cfg->pr;
    double pinf = 1.0 / (cfg->gamma * cfg->mach * cfg->mach);
    c->Uinf[0] = 1.0; c->Uinf[1] = 1.0; c->Uinf[2] = 0.0;
    c->Uinf[3] = pinf / (cfg->gamma - 1.0) + 0.5;
    double A[9], bw[3], cc[3];
    pao_dirk_tableau(A, bw, cc);
    for (int i = 0; i < 3; ++i) { c->bw[i] = bw[i]; c->cc[i] = cc[i]; for (int j = 0; j < 3; ++j) c->A[i][j] = A[3 * i + j]; }
    c->dt = cfg->T / cfg->Nt;
    return c;
}

void pao_destroy(pao_ctx* c)
{
    if (!c) return;
    void* ptrs[] = { c->vxy, c->ev, c->enb, c->etw, c->area, c->jit, c->xn, c->wbl, c->rn, c->mx, c->my, c->C,
                     c->xq, c->wq, c->phq, c->dphq, c->sf, c->wf, c->phf, c->dphf, c->phfr, c->dphfr, c->mh,
                     c->mhi, c->gb[0], c->gb[1], c->gb[2], c->gb[3], c->tu, c->tk, c->tui, c->tJ };
    for (size_t k = 0; k < sizeof ptrs / sizeof ptrs[0]; ++k) free(ptrs[k]);
    free(c);
}

const char* pao_last_error(const pao_ctx* c) { return c ? c->err : "null context"; }
int64_t pao_num_dofs(const pao_ctx* c) { return c->Nu; }
int32_t pao_num_elems(const pao_ctx* c) { return c->Ne; }
int32_t pao_block_size(const pao_ctx* c) { return c->b; }
int32_t pao_num_vol_points(const pao_ctx* c) { return c->nq; }

void pao_get_mesh(const pao_ctx* c, int32_t* ev, int32_t* en, int8_t* tw, double* vxy)
{
    if (ev) memcpy(ev, c->ev, sizeof(int32_t) * c->Ne * 3);
    if (en) memcpy(en, c->enb, sizeof(int32_t) * c->Ne * 3);
    if (tw) memcpy(tw, c->etw, sizeof(int8_t) * c->Ne * 3);
    if (vxy) memcpy(vxy, c->vxy, sizeof(double) * c->nv * 2);
}

void pao_get_nodes(const pao_ctx* c, double* xn, double* area)
{
    if (xn) memcpy(xn, c->xn, sizeof(double) * c->Ne * c->np * 2);
    if (area) memcpy(area, c->area, sizeof(double) * c->Ne);
}

void pao_ref_tables(const pao_ctx* c, double* xq, double* wq, double* phq, double* mh)
{
    if (xq) memcpy(xq, c->xq, sizeof(double) * c->nq * 2);
    if (wq) memcpy(wq, c->wq, sizeof(double) * c->nq);
    if (phq) memcpy(phq, c->phq, sizeof(double) * c->nq * c->np);
    if (mh) memcpy(mh, c->mh, sizeof(double) * c->np * c->np);
}

int pao_set_params(pao_ctx* c, const double mu[3])
{
    memcpy(c->mu, mu, sizeof(double) * 3);
    int64_t nn = (int64_t)c->Ne * c->np * (c->nst + 1);
    if (!c->gb[0]) c->gb[0] = malloc(sizeof(cplx) * nn);
    cplx m[3] = { mu[0], mu[1], mu[2] };
    gbar_compute(c, m, c->gb[0]);
    c->have_params = 1;
    c->have_dgb = 0;
    c->have_traj = 0;
    return 0;
}

int pao_gbar(pao_ctx* c, int32_t n, int32_t i, double* out)
{
    int rc = check_stage(c, n, i);
    if (rc) return rc;
    int64_t nn = (int64_t)c->Ne * c->np;
    const cplx* g = c->gb[0] + (int64_t)stage_index(n, i) * nn;
    for (int64_t k = 0; k < nn; ++k) out[k] = creal(g[k]);
    return 0;
}

int pao_gcl_rhs(pao_ctx* c, int32_t n, int32_t i, double* out)
{
    int rc = check_stage(c, n, i);
    if (rc) return rc;
    Motion m;
    motion_alloc(c, &m);
    Stage S = stage_make(c, n, i, 0, &m);
    int64_t nn = (int64_t)c->Ne * c->np;
    cplx* rg = malloc(sizeof(cplx) * nn);
    gcl_rhs_all(c, &S, rg);
    for (int64_t k = 0; k < nn; ++k) out[k] = creal(rg[k]);
    free(rg);
    motion_free(&m);
    return 0;
}

int pao_freestream(pao_ctx* c, const double* pert, double* u)
{
    if (!c->gb[0]) return -1;   /* the parameters (and with them gbar at t = 0) are not set yet */
    int np = c->np;
    for (int K = 0; K < c->Ne; ++K)
        for (int a = 0; a < np; ++a) {
            double g = creal(c->gb[0][(int64_t)K * np + a]);
            for (int m = 0; m < 4; ++m) {
                int64_t idx = ((int64_t)K * np + a) * 4 + m;
                u[idx] = g * c->Uinf[m] + (pert ? pert[idx] : 0.0);
            }
        }
    return 0;
}

int pao_residual(pao_ctx* c, int32_t n, int32_t i, const double* u, double* r)
{
    int rc = check_stage(c, n, i);
    if (rc) return rc;
    Motion m;
    motion_alloc(c, &m);
    Stage S = stage_make(c, n, i, 0, &m);
    cplx* uc = to_cplx(c, u);
    residual_stage(c, &S, uc, r, NULL);
    free(uc);
    motion_free(&m);
    return 0;
}

int pao_jacobian(pao_ctx* c, int32_t n, int32_t i, const double* u, double* blk)
{
    int rc = check_stage(c, n, i);
    if (rc) return rc;
    Motion m;
    motion_alloc(c, &m);
    Stage S = stage_make(c, n, i, 0, &m);
    jacobian_stage(c, &S, u, blk);
    motion_free(&m);
    return 0;
}

int pao_dr_dmu(pao_ctx* c, int32_t n, int32_t i, const double* u, double* out)
{
    int rc = check_stage(c, n, i);
    if (rc) return rc;
    drdmu_stage(c, n, i, u, out);
    return 0;
}

int pao_qoi(pao_ctx* c, int32_t n, int32_t i, const double* u, double f[2], double* dfdu, double* dfdmu)
{
    int rc = check_stage(c, n, i);
    if (rc) return rc;
    qoi_stage(c, n, i, u, f, dfdu, dfdmu);
    return 0;
}

static int finite_vec(int64_t n, const double* x)
{
    for (int64_t k = 0; k < n; ++k) if (!isfinite(x[k])) return 0;
    return 1;
}

/* ------------------------------------------------------------------ */
/* sweeps                                                               */
/* ------------------------------------------------------------------ */
static int traj_alloc(pao_ctx* c)
{
    int64_t Nu = c->Nu;
    if (!c->tu) {
        c->tu = malloc(sizeof(double) * Nu * (c->Nt + 1));
        c->tk = malloc(sizeof(double) * Nu * c->nst);
        c->tui = malloc(sizeof(double) * Nu * c->nst);
        c->tJ = malloc(sizeof(double) * (size_t)c->Ne * 4 * c->b * c->b * c->nst);
        if (!c->tu || !c->tk || !c->tui || !c->tJ) return fail(c, -1, "out of memory for trajectory");
    }
    return 0;
}

#define JSZ(c) ((int64_t)(c)->Ne * 4 * (c)->b * (c)->b)

/* Primal period (eq. dirk2): per stage, Newton on
 *   R_i(k) = M k - dt r(u^(n-1) + sum_{j<i} a_ij k_j + a_ii k)
 * with the exact Jacobian M - dt a_ii dr/du and backtracking halving;
 * predictor k_i <- previous stage's k.  After convergence the Jacobian at
 * the converged stage state is stored for the tangent and adjoint sweeps. */
int pao_primal_period(pao_ctx* c, const double* u0, double* uNt, double qoi[2], double* res)
{
    if (!c->have_params) return fail(c, -4, "parameters not set");
    int rc = traj_alloc(c);
    if (rc) return rc;
    if (!finite_vec(c->Nu, u0)) return fail(c, -3, "non-finite initial state");
    int64_t Nu = c->Nu;
    double *ubase = malloc(sizeof(double) * Nu), *k = calloc(Nu, sizeof(double)), *ui = malloc(sizeof(double) * Nu);
    double *R = malloc(sizeof(double) * Nu), *r = malloc(sizeof(double) * Nu), *dk = malloc(sizeof(double) * Nu);
    double *kt = malloc(sizeof(double) * Nu), *Jt = malloc(sizeof(double) * JSZ(c));
    memcpy(c->tu, u0, sizeof(double) * Nu);
    double Jq[2] = { 0, 0 };
    c->cnt_newton = 0;
    c->cnt_lin = 0;
    rc = 0;
    for (int n = 1; n <= c->Nt && !rc; ++n) {
        const double* uprev = c->tu + (int64_t)(n - 1) * Nu;
        for (int i = 1; i <= 3 && !rc; ++i) {
            int s = (n - 1) * 3 + (i - 1);
            for (int64_t q = 0; q < Nu; ++q) {
                double acc = uprev[q];
                for (int j = 1; j < i; ++j) acc += c->A[i - 1][j - 1] * c->tk[(int64_t)(s - i + j) * Nu + q];
                ubase[q] = acc;
            }
            double aii = c->A[i - 1][i - 1];
#define EVAL_R(kk, out_norm)                                                         \
    do {                                                                             \
        for (int64_t q = 0; q < Nu; ++q) ui[q] = ubase[q] + aii * (kk)[q];          \
        pao_residual(c, n, i, ui, r);                                                \
        pao_mass_apply(c, (kk), R);                                                  \
        for (int64_t q = 0; q < Nu; ++q) R[q] -= c->dt * r[q];                       \
        out_norm = nrm2(Nu, R);                                                      \
    } while (0)
            /* predictor (reading; the paper fixes none): the previous stage's
             * slope k_{i-1}, or the slope that puts u_i at the previous stage
             * state; the one with the smaller Newton residual is kept (the
             * slope on ties).  The first stage of the period starts from 0. */
            double nR;
            if (s > 0) {
                const double* uprv = c->tui + (int64_t)(s - 1) * Nu;
                double n2;
                for (int64_t q = 0; q < Nu; ++q) kt[q] = (uprv[q] - ubase[q]) / aii;
                EVAL_R(kt, n2);
                memcpy(k, c->tk + (int64_t)(s - 1) * Nu, sizeof(double) * Nu);
                EVAL_R(k, nR);
                if (!(nR <= n2)) { memcpy(k, kt, sizeof(double) * Nu); EVAL_R(k, nR); }
            } else {
                memset(k, 0, sizeof(double) * Nu);
                EVAL_R(k, nR);
            }
            int it = 0;
            while (!(nR <= c->cfg.newton_atol)) {
                if (!isfinite(nR)) { rc = fail(c, -3, "NaN in stage (%d,%d)", n, i); break; }
                if (it >= c->cfg.newton_maxit) {
                    rc = fail(c, -2, "Newton did not converge at stage (%d,%d): |R| = %.3e", n, i, nR);
                    break;
                }
                pao_jacobian(c, n, i, ui, Jt);
                int li = pao_stage_solve(c, Jt, c->dt * aii, 0, R, dk);
                if (li < 0) { rc = li; break; }
                /* backtracking: halve until ||R|| decreases (NaN counts as no decrease) */
                double lam = 1.0, nT = 0;
                for (;;) {
                    for (int64_t q = 0; q < Nu; ++q) kt[q] = k[q] - lam * dk[q];
                    EVAL_R(kt, nT);
                    if (nT < nR) break;
                    lam *= 0.5;
                    if (lam < 1e-4) { rc = fail(c, -2, "line search failed at stage (%d,%d)", n, i); break; }
                }
                if (rc) break;
                memcpy(k, kt, sizeof(double) * Nu);
                nR = nT;
                ++it;
                ++c->cnt_newton;
            }
#undef EVAL_R
            if (rc) break;
            for (int64_t q = 0; q < Nu; ++q) ui[q] = ubase[q] + aii * k[q];
            memcpy(c->tk + (int64_t)s * Nu, k, sizeof(double) * Nu);
            memcpy(c->tui + (int64_t)s * Nu, ui, sizeof(double) * Nu);
            pao_jacobian(c, n, i, ui, c->tJ + (int64_t)s * JSZ(c));
            double f[2];
            qoi_stage(c, n, i, ui, f, NULL, NULL);
            Jq[0] += c->dt * c->bw[i - 1] * f[0] / c->cfg.T;
            Jq[1] += c->dt * c->bw[i - 1] * f[1] / c->cfg.T;
        }
        if (rc) break;
        double* un = c->tu + (int64_t)n * Nu;
        for (int64_t q = 0; q < Nu; ++q) {
            double acc = uprev[q];
            for (int i = 0; i < 3; ++i) acc += c->bw[i] * c->tk[(int64_t)((n - 1) * 3 + i) * Nu + q];
            un[q] = acc;
        }
    }
    free(ubase); free(k); free(ui); free(R); free(r); free(dk); free(kt); free(Jt);
    if (rc) { c->have_traj = 0; return rc; }
    c->have_traj = 1;
    const double* un = c->tu + (int64_t)c->Nt * Nu;
    if (uNt) memcpy(uNt, un, sizeof(double) * Nu);
    if (qoi) { qoi[0] = Jq[0]; qoi[1] = Jq[1]; }
    if (res) {
        double s = 0;
        for (int64_t q = 0; q < Nu; ++q) s += (un[q] - u0[q]) * (un[q] - u0[q]);
        *res = sqrt(s);
    }
    return 0;
}

/* Tangent sweep (eq. dirk-sens-mvp in the stage form):
 *   (M - dt a_ii J_i) dk_i = dt J_i (du^(n-1) + sum_{j<i} a_ij dk_j) [+ dt dr/dmu_k]
 *   du^(n) = du^(n-1) + sum_i b_i dk_i */
int pao_tangent_sweep(pao_ctx* c, const double* v, int32_t mu_dir, double* out, double* dqoi)
{
    if (!c->have_traj) return fail(c, -4, "no primal trajectory");
    int64_t Nu = c->Nu;
    double *du = malloc(sizeof(double) * Nu), *dk = malloc(sizeof(double) * Nu * 3);
    double *w = malloc(sizeof(double) * Nu), *rhs = malloc(sizeof(double) * Nu), *dr = NULL, *df = NULL;
    if (mu_dir >= 0) dr = malloc(sizeof(double) * Nu * 3);
    if (dqoi) df = malloc(sizeof(double) * Nu * 2);
    memcpy(du, v, sizeof(double) * Nu);
    double dq[2] = { 0, 0 };
    int rc = 0;
    for (int n = 1; n <= c->Nt && !rc; ++n) {
        for (int i = 1; i <= 3; ++i) {
            int s = (n - 1) * 3 + (i - 1);
            const double* J = c->tJ + (int64_t)s * JSZ(c);
            for (int64_t q = 0; q < Nu; ++q) {
                double acc = du[q];
                for (int j = 1; j < i; ++j) acc += c->A[i - 1][j - 1] * dk[(int64_t)(j - 1) * Nu + q];
                w[q] = acc;
            }
            pao_bsr_apply(c, J, 0, w, rhs);
            for (int64_t q = 0; q < Nu; ++q) rhs[q] *= c->dt;
            if (mu_dir >= 0) {
                drdmu_stage(c, n, i, c->tui + (int64_t)s * Nu, dr);
                for (int64_t q = 0; q < Nu; ++q) rhs[q] += c->dt * dr[(int64_t)mu_dir * Nu + q];
            }
            double* dki = dk + (int64_t)(i - 1) * Nu;
            int li = pao_stage_solve(c, J, c->dt * c->A[i - 1][i - 1], 0, rhs, dki);
            if (li < 0) { rc = li; break; }
            if (dqoi) {
                double f[2], fm[6];
                qoi_stage(c, n, i, c->tui + (int64_t)s * Nu, f, df, mu_dir >= 0 ? fm : NULL);
                /* d u_i = w + a_ii dk_i */
                for (int qq = 0; qq < 2; ++qq) {
                    double acc = 0;
                    for (int64_t q = 0; q < Nu; ++q) acc += df[qq * Nu + q] * (w[q] + c->A[i - 1][i - 1] * dki[q]);
                    if (mu_dir >= 0) acc += fm[3 * qq + mu_dir];
                    dq[qq] += c->dt * c->bw[i - 1] * acc / c->cfg.T;
                }
            }
        }
        if (rc) break;
        for (int64_t q = 0; q < Nu; ++q)
            du[q] += c->bw[0] * dk[q] + c->bw[1] * dk[Nu + q] + c->bw[2] * dk[2 * Nu + q];
    }
    if (!rc) { memcpy(out, du, sizeof(double) * Nu); if (dqoi) { dqoi[0] = dq[0]; dqoi[1] = dq[1]; } }
    free(du); free(dk); free(w); free(rhs); free(dr); free(df);
    return rc;
}

/* Backward adjoint sweep (eqs. uns-disc-adj-dirk2 / uns-disc-adj-dirk-sens-mvp):
 *   (M - dt a_ii J_i)^T kappa_i = dF/dk_i + b_i lambda^(n) + sum_{j>i} a_ji dt J_j^T kappa_j
 *   lambda^(n-1) = lambda^(n) + dF/du^(n-1) + sum_i dt J_i^T kappa_i
 * and, when forced, dF/dmu = dF/dmu|explicit + sum dt kappa_i^T dr/dmu(u_i)
 * (eq. funcl-grad-nosens-dirk).  For the time-averaged QoI
 *   F = (1/T) sum_n sum_i dt b_i f(u_i^(n))
 * one has dF/du^(n-1) = (1/T) sum_i dt b_i f_i', dF/dk_j = (1/T) sum_{i>=j} dt b_i a_ij f_i'. */
int pao_adjoint_sweep(pao_ctx* c, const double* lamNt, int32_t fq, double* lam0, double* grad)
{
    if (!c->have_traj) return fail(c, -4, "no primal trajectory");
    int64_t Nu = c->Nu;
    double *lam = malloc(sizeof(double) * Nu), *z = malloc(sizeof(double) * Nu * 3);
    double *kap = malloc(sizeof(double) * Nu), *rhs = malloc(sizeof(double) * Nu);
    double *fp = NULL, *dr = NULL;
    if (fq >= 0) { fp = malloc(sizeof(double) * Nu * 3 * 2); dr = malloc(sizeof(double) * Nu * 3); }
    memcpy(lam, lamNt, sizeof(double) * Nu);
    double g[3] = { 0, 0, 0 };
    double sc = c->dt / c->cfg.T;
    int rc = 0;
    for (int n = c->Nt; n >= 1 && !rc; --n) {
        if (fq >= 0)
            for (int i = 1; i <= 3; ++i) {
                int s = (n - 1) * 3 + (i - 1);
                double f[2], fm[6], *dfdu = malloc(sizeof(double) * Nu * 2);
                qoi_stage(c, n, i, c->tui + (int64_t)s * Nu, f, dfdu, fm);
                memcpy(fp + (int64_t)(i - 1) * Nu, dfdu + (int64_t)fq * Nu, sizeof(double) * Nu);
                free(dfdu);
                for (int k = 0; k < 3; ++k) g[k] += sc * c->bw[i - 1] * fm[3 * fq + k];
            }
        for (int i = 3; i >= 1; --i) {
            int s = (n - 1) * 3 + (i - 1);
            const double* J = c->tJ + (int64_t)s * JSZ(c);
            for (int64_t q = 0; q < Nu; ++q) {
                double acc = c->bw[i - 1] * lam[q];
                for (int j = i + 1; j <= 3; ++j) acc += c->A[j - 1][i - 1] * z[(int64_t)(j - 1) * Nu + q];
                if (fq >= 0)
                    for (int j = i; j <= 3; ++j) acc += sc * c->bw[j - 1] * c->A[j - 1][i - 1] * fp[(int64_t)(j - 1) * Nu + q];
                rhs[q] = acc;
            }
            int li = pao_stage_solve(c, J, c->dt * c->A[i - 1][i - 1], 1, rhs, kap);
            if (li < 0) { rc = li; break; }
            double* zi = z + (int64_t)(i - 1) * Nu;
            pao_bsr_apply(c, J, 1, kap, zi);
            for (int64_t q = 0; q < Nu; ++q) zi[q] *= c->dt;
            if (fq >= 0) {
                drdmu_stage(c, n, i, c->tui + (int64_t)s * Nu, dr);
                for (int k = 0; k < 3; ++k) g[k] += c->dt * dot(Nu, kap, dr + (int64_t)k * Nu);
            }
        }
        if (rc) break;
        for (int64_t q = 0; q < Nu; ++q) {
            double acc = lam[q] + z[q] + z[Nu + q] + z[2 * Nu + q];
            if (fq >= 0) for (int i = 0; i < 3; ++i) acc += sc * c->bw[i] * fp[(int64_t)i * Nu + q];
            lam[q] = acc;
        }
    }
    if (!rc) { memcpy(lam0, lam, sizeof(double) * Nu); if (grad) memcpy(grad, g, sizeof g); }
    free(lam); free(z); free(kap); free(rhs); free(fp); free(dr);
    return rc;
}

/* matrix-free operators for the outer Krylov solves */
typedef struct { pao_ctx* c; int rc; } OuterOp;

static void op_phi_minus_I(void* ctx, const double* v, double* w)
{
    OuterOp* o = ctx;
    if (o->rc) { memset(w, 0, sizeof(double) * o->c->Nu); return; }
    int rc = pao_tangent_sweep(o->c, v, -1, w, NULL);
    if (rc) { o->rc = rc; return; }
    for (int64_t q = 0; q < o->c->Nu; ++q) w[q] -= v[q];
}

static void op_phiT_minus_I(void* ctx, const double* v, double* w)
{
    OuterOp* o = ctx;
    if (o->rc) { memset(w, 0, sizeof(double) * o->c->Nu); return; }
    int rc = pao_adjoint_sweep(o->c, v, -1, w, NULL);
    if (rc) { o->rc = rc; return; }
    for (int64_t q = 0; q < o->c->Nu; ++q) w[q] -= v[q];
}

/* Newton-Krylov shooting (Alg. 2, read with the Jacobian Phi - I of eq.
 * jac-prim): solve (Phi - I) D = R with matrix-free GMRES, u0 <- u0 - D */
int pao_shoot(pao_ctx* c, double* u0, double tol, double eta, int32_t maxit, int32_t max_krylov,
              pao_krylov_report* rep)
{
    int64_t Nu = c->Nu;
    double *uNt = malloc(sizeof(double) * Nu), *R = malloc(sizeof(double) * Nu), *D = malloc(sizeof(double) * Nu);
    pao_krylov_report r = { 0, 0, 0, 0 };
    int rc = 0;
    for (;;) {
        double qoi[2], res;
        rc = pao_primal_period(c, u0, uNt, qoi, &res);
        ++r.sweeps;
        if (rc) break;
        r.final_res = res;
        if (res <= tol) break;
        if (r.outer_its >= maxit) { rc = fail(c, -2, "shooting did not converge: |R| = %.3e", res); break; }
        for (int64_t q = 0; q < Nu; ++q) R[q] = uNt[q] - u0[q];
        OuterOp o = { c, 0 };
        double rr;
        int its = gmres(Nu, op_phi_minus_I, NULL, &o, R, D, eta, max_krylov, max_krylov, &rr);
        if (o.rc) { rc = o.rc; break; }
        if (its < 0) its = max_krylov;   /* inexact Newton: accept the last iterate */
        r.krylov_its += its;
        r.sweeps += its + 1;
        for (int64_t q = 0; q < Nu; ++q) u0[q] -= D[q];
        ++r.outer_its;
    }
    free(uNt); free(R); free(D);
    if (rep) *rep = r;
    return rc;
}

/* Periodic adjoint (Alg. 3 and Alg. 4): with g_F the forced backward sweep
 * from lambda_Nt = 0, solve (Phi^T - I) lambda_Nt = -(g_F + dF/du^(Nt)^T)
 * (dF/du^(Nt) = 0 for the time-averaged QoIs), then one forced sweep from
 * lambda_Nt gives the gradient. */
int pao_periodic_adjoint(pao_ctx* c, int32_t q, double rtol, int32_t max_krylov, double* lamNt, double* grad,
                         pao_krylov_report* rep)
{
    int64_t Nu = c->Nu;
    double *zero = calloc(Nu, sizeof(double)), *gF = malloc(sizeof(double) * Nu), *l0 = malloc(sizeof(double) * Nu);
    pao_krylov_report r = { 1, 0, 0, 0 };
    int rc = pao_adjoint_sweep(c, zero, q, gF, NULL);
    r.sweeps = 1;
    if (!rc) {
        for (int64_t k = 0; k < Nu; ++k) gF[k] = -gF[k];
        OuterOp o = { c, 0 };
        double rr;
        int its = gmres(Nu, op_phiT_minus_I, NULL, &o, gF, lamNt, rtol, max_krylov, max_krylov, &rr);
        if (o.rc) rc = o.rc;
        else if (its < 0) rc = fail(c, -2, "periodic adjoint GMRES did not converge (%.3e)", rr);
        else {
            r.krylov_its = its;
            r.sweeps += its + 1;
            r.final_res = rr;
            rc = pao_adjoint_sweep(c, lamNt, q, l0, grad);
            r.sweeps += 1;
        }
    }
    free(zero); free(gF); free(l0);
    if (rep) *rep = r;
    return rc;
}

/* Direct gradient: for each mu_k, periodic tangent (Phi - I) du0 = -s_k with
 * s_k the mu_k-forced tangent sweep from 0, then the QoI tangent of the
 * forced sweep from du0. */
int pao_tangent_gradient(pao_ctx* c, double rtol, int32_t max_krylov, double* dJ)
{
    int64_t Nu = c->Nu;
    double *zero = calloc(Nu, sizeof(double)), *s = malloc(sizeof(double) * Nu), *du0 = malloc(sizeof(double) * Nu);
    double *tmp = malloc(sizeof(double) * Nu);
    int rc = 0;
    for (int k = 0; k < 3 && !rc; ++k) {
        rc = pao_tangent_sweep(c, zero, k, s, NULL);
        if (rc) break;
        for (int64_t q = 0; q < Nu; ++q) s[q] = -s[q];
        OuterOp o = { c, 0 };
        double rr;
        int its = gmres(Nu, op_phi_minus_I, NULL, &o, s, du0, rtol, max_krylov, max_krylov, &rr);
        if (o.rc) { rc = o.rc; break; }
        if (its < 0) { rc = fail(c, -2, "tangent GMRES did not converge"); break; }
        double dq[2];
        rc = pao_tangent_sweep(c, du0, k, tmp, dq);
        dJ[k] = dq[0];
        dJ[3 + k] = dq[1];
    }
    free(zero); free(s); free(du0); free(tmp);
    return rc;
}

int pao_traj(pao_ctx* c, int32_t which, int32_t n, int32_t i, double* out)
{
    if (!c->have_traj) return fail(c, -4, "no trajectory");
    int64_t Nu = c->Nu;
    if (which == 2) {
        if (n < 0 || n > c->Nt) return fail(c, -1, "bad step");
        memcpy(out, c->tu + (int64_t)n * Nu, sizeof(double) * Nu);
        return 0;
    }
    if (n < 1 || n > c->Nt || i < 1 || i > 3) return fail(c, -1, "bad stage");
    int s = (n - 1) * 3 + (i - 1);
    memcpy(out, (which == 0 ? c->tui : c->tk) + (int64_t)s * Nu, sizeof(double) * Nu);
    return 0;
}

int pao_traj_jacobian(pao_ctx* c, int32_t n, int32_t i, double* blk)
{
    if (!c->have_traj) return fail(c, -4, "no trajectory");
    if (n < 1 || n > c->Nt || i < 1 || i > 3) return fail(c, -1, "bad stage");
    int s = (n - 1) * 3 + (i - 1);
    memcpy(blk, c->tJ + (int64_t)s * JSZ(c), sizeof(double) * JSZ(c));
    return 0;
}

/* ------------------------------------------------------------------ */
/* test hooks: the pointwise fluxes and the face lifting                 */
/* ------------------------------------------------------------------ */
void pao_flux_vis(const pao_ctx* c, const double U[4], const double dU[8], int32_t heat, double F[8])
{
    cplx Uc[4], dUc[4][2], Fc[4][2];
    for (int m = 0; m < 4; ++m) {
        Uc[m] = U[m];
        dUc[m][0] = dU[2 * m];
        dUc[m][1] = dU[2 * m + 1];
    }
    flux_vis(c, Uc, dUc, Fc, heat);
    for (int m = 0; m < 4; ++m) {
        F[2 * m] = creal(Fc[m][0]);
        F[2 * m + 1] = creal(Fc[m][1]);
    }
}

void pao_flux_h(const pao_ctx* c, const double U[4], const double n[2], double vn, double H[4])
{
    cplx Uc[4] = { U[0], U[1], U[2], U[3] }, nc[2] = { n[0], n[1] }, Hc[4];
    flux_H(c, Uc, nc, vn, Hc);
    for (int m = 0; m < 4; ++m) H[m] = creal(Hc[m]);
}

void pao_flux_lf(const pao_ctx* c, const double UL[4], const double UR[4], const double n[2], double vn, double F[4])
{
    cplx L[4] = { UL[0], UL[1], UL[2], UL[3] }, R[4] = { UR[0], UR[1], UR[2], UR[3] }, nc[2] = { n[0], n[1] }, Fc[4];
    flux_lf(c, L, R, nc, vn, Fc);
    for (int m = 0; m < 4; ++m) F[m] = creal(Fc[m]);
}

int pao_face_lift(pao_ctx* c, int32_t n, int32_t i, const double* u, int32_t K, int32_t f, double* lift)
{
    int rc = check_stage(c, n, i);
    if (rc) return rc;
    if (K < 0 || K >= c->Ne || f < 0 || f > 2) return fail(c, -1, "bad face (%d, %d)", K, f);
    int nb = c->enb[3 * K + f];
    if (nb < 0) return fail(c, -1, "face (%d, %d) is on the boundary", K, f);
    int tw = c->etw[3 * K + f];
    int L, fL, R, fR;
    if (K < nb) { L = K; fL = f; R = nb; fR = tw; }
    else { L = nb; fL = tw; R = K; fR = f; }
    Motion m;
    motion_alloc(c, &m);
    Stage S = stage_make(c, n, i, 0, &m);
    cplx* uc = to_cplx(c, u);
    cplx Fh[8 * 4], lf[16 * 8];
    face_interior(c, &S, L, fL, R, fR, uc, Fh, lf);
    for (int k = 0; k < c->np * 8; ++k) lift[k] = creal(lf[k]);
    free(uc);
    motion_free(&m);
    return K == L ? 1 : 0;
}

void pao_counters(const pao_ctx* c, int64_t* newton, int64_t* linear)
{
    if (newton) *newton = c->cnt_newton;
    if (linear) *linear = c->cnt_lin;
}
