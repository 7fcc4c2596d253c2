// Device-side arithmetic for the periodic-adjoint HIP library (gfx950).
//
// * forward-mode dual numbers (exact pointwise Jacobians and mu-derivatives)
// * compressible Navier-Stokes fluxes (arXiv:1512.00616 Sec. 4, eqs. ns1-ns5)
//   and their ALE pull-back to the fixed reference domain (eqs. ns-cons-ref,
//   transform1-nogcl, transform2-nogcl) with the GCL-consistent factor gbar
// * the numerical fluxes and boundary conditions of the discretisation
//
// Every routine is a template on the scalar type T (double, Dual<1>, Dual<3>)
// so that one source gives values, state Jacobians and parameter derivatives.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pa {

// ------------------------------------------------------------------ dual numbers
template <int N>
struct Dual {
    double v;
    double d[N];
};

template <class T>
struct AD;
template <>
struct AD<double> {
    static __device__ __host__ __forceinline__ double c(double x) { return x; }
    static __device__ __host__ __forceinline__ double val(double x) { return x; }
};
template <int N>
struct AD<Dual<N>> {
    static __device__ __host__ __forceinline__ Dual<N> c(double x)
    {
        Dual<N> r;
        r.v = x;
#pragma unroll
        for (int i = 0; i < N; ++i) r.d[i] = 0.0;
        return r;
    }
    static __device__ __host__ __forceinline__ double val(const Dual<N>& x) { return x.v; }
};

#define PA_DUAL_BINOP(OP, VEXPR, DEXPR)                                                           \
    template <int N>                                                                              \
    __device__ __host__ __forceinline__ Dual<N> operator OP(const Dual<N>& a, const Dual<N>& b)   \
    {                                                                                             \
        Dual<N> r;                                                                                \
        r.v = VEXPR;                                                                              \
        _Pragma("unroll") for (int i = 0; i < N; ++i) r.d[i] = DEXPR;                             \
        return r;                                                                                 \
    }
PA_DUAL_BINOP(+, a.v + b.v, a.d[i] + b.d[i])
PA_DUAL_BINOP(-, a.v - b.v, a.d[i] - b.d[i])
PA_DUAL_BINOP(*, a.v * b.v, a.d[i] * b.v + a.v * b.d[i])
#undef PA_DUAL_BINOP

template <int N>
__device__ __host__ __forceinline__ Dual<N> operator/(const Dual<N>& a, const Dual<N>& b)
{
    Dual<N> r;
    double ib = 1.0 / b.v;
    r.v = a.v * ib;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) * ib;
    return r;
}
template <int N>
__device__ __host__ __forceinline__ Dual<N> operator-(const Dual<N>& a)
{
    Dual<N> r;
    r.v = -a.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = -a.d[i];
    return r;
}
template <int N>
__device__ __host__ __forceinline__ Dual<N> operator*(const Dual<N>& a, double s)
{
    Dual<N> r;
    r.v = a.v * s;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * s;
    return r;
}
template <int N>
__device__ __host__ __forceinline__ Dual<N> operator*(double s, const Dual<N>& a) { return a * s; }
template <int N>
__device__ __host__ __forceinline__ Dual<N> operator+(const Dual<N>& a, double s)
{
    Dual<N> r = a;
    r.v += s;
    return r;
}
template <int N>
__device__ __host__ __forceinline__ Dual<N> operator+(double s, const Dual<N>& a) { return a + s; }
template <int N>
__device__ __host__ __forceinline__ Dual<N> operator-(const Dual<N>& a, double s)
{
    Dual<N> r = a;
    r.v -= s;
    return r;
}
template <int N>
__device__ __host__ __forceinline__ Dual<N> operator-(double s, const Dual<N>& a)
{
    Dual<N> r = -a;
    r.v += s;
    return r;
}
template <int N>
__device__ __host__ __forceinline__ Dual<N> operator/(const Dual<N>& a, double s) { return a * (1.0 / s); }
template <int N>
__device__ __host__ __forceinline__ Dual<N> operator/(double s, const Dual<N>& b)
{
    Dual<N> r;
    double ib = 1.0 / b.v;
    r.v = s * ib;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = -r.v * b.d[i] * ib;
    return r;
}
template <int N>
__device__ __host__ __forceinline__ Dual<N>& operator+=(Dual<N>& a, const Dual<N>& b) { a = a + b; return a; }
template <int N>
__device__ __host__ __forceinline__ Dual<N>& operator-=(Dual<N>& a, const Dual<N>& b) { a = a - b; return a; }
template <int N>
__device__ __host__ __forceinline__ Dual<N>& operator+=(Dual<N>& a, double b) { a.v += b; return a; }

__device__ __host__ __forceinline__ double dsqrt(double x) { return sqrt(x); }
template <int N>
__device__ __host__ __forceinline__ Dual<N> dsqrt(const Dual<N>& a)
{
    Dual<N> r;
    r.v = sqrt(a.v);
    double s = 0.5 / r.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * s;
    return r;
}
__device__ __host__ __forceinline__ void dsincos(double a, double* s, double* c)
{
    *s = sin(a);
    *c = cos(a);
}
template <int N>
__device__ __host__ __forceinline__ void dsincos(const Dual<N>& a, Dual<N>* s, Dual<N>* c)
{
    double sv = sin(a.v), cv = cos(a.v);
    s->v = sv;
    c->v = cv;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        s->d[i] = cv * a.d[i];
        c->d[i] = -sv * a.d[i];
    }
}

// ------------------------------------------------------------------ physics
struct Phys {
    double gam, muv, pr;   // ratio of specific heats, viscosity 1/Re, Prandtl number
    double Uinf[4];        // free-stream conserved state
    double lf_delta;       // smoothing of |u.n - v.n| in the dissipation speed
    double wall_eta;       // wall penalty C11 = wall_eta / h
};

// inviscid flux F_inv(U), F[m][d]
template <class T>
__device__ __forceinline__ void flux_inv(const Phys& ph, const T U[4], T F[4][2])
{
    T ir = 1.0 / U[0];
    T ux = U[1] * ir, uy = U[2] * ir;
    T p = (ph.gam - 1.0) * (U[3] - 0.5 * (U[1] * ux + U[2] * uy));
    F[0][0] = U[1];
    F[0][1] = U[2];
    F[1][0] = U[1] * ux + p;
    F[1][1] = U[1] * uy;
    F[2][0] = U[2] * ux;
    F[2][1] = U[2] * uy + p;
    T e = U[3] + p;
    F[3][0] = e * ux;
    F[3][1] = e * uy;
}

// viscous flux F_vis(U, dU) with dU the physical gradient dU[m][d];
// heat == false drops the heat flux (adiabatic wall)
template <class T>
__device__ __forceinline__ void flux_vis(const Phys& ph, const T U[4], const T dU[4][2], T F[4][2], bool heat)
{
    T ir = 1.0 / U[0];
    T u0 = U[1] * ir, u1 = U[2] * ir, E = U[3] * ir;
    T du[2][2], dE[2];
#pragma unroll
    for (int d = 0; d < 2; ++d) {
        du[0][d] = (dU[1][d] - u0 * dU[0][d]) * ir;
        du[1][d] = (dU[2][d] - u1 * dU[0][d]) * ir;
        dE[d] = (dU[3][d] - E * dU[0][d]) * ir;
    }
    T div = du[0][0] + du[1][1];
    T t00 = ph.muv * (2.0 * du[0][0] - (2.0 / 3.0) * div);
    T t11 = ph.muv * (2.0 * du[1][1] - (2.0 / 3.0) * div);
    T t01 = ph.muv * (du[0][1] + du[1][0]);
    double kap = ph.muv / ph.pr * ph.gam;   // q = -(mu/Pr) grad(gamma (E - |u|^2/2))
    F[0][0] = AD<T>::c(0.0);
    F[0][1] = AD<T>::c(0.0);
    F[1][0] = t00;
    F[1][1] = t01;
    F[2][0] = t01;
    F[2][1] = t11;
#pragma unroll
    for (int d = 0; d < 2; ++d) {
        T tw = (d == 0) ? (u0 * t00 + u1 * t01) : (u0 * t01 + u1 * t11);
        if (heat)
            F[3][d] = tw + kap * (dE[d] - u0 * du[0][d] - u1 * du[1][d]);
        else
            F[3][d] = tw;
    }
}

// H(U) = F_inv(U) n - U (v_G . n)
template <class T>
__device__ __forceinline__ void flux_H(const Phys& ph, const T U[4], const T n[2], const T& vn, T H[4])
{
    T F[4][2];
    flux_inv(ph, U, F);
#pragma unroll
    for (int m = 0; m < 4; ++m) H[m] = F[m][0] * n[0] + F[m][1] * n[1] - U[m] * vn;
}

template <class T>
__device__ __forceinline__ T wave_speed(const Phys& ph, const T U[4], const T n[2], const T& vn)
{
    T ir = 1.0 / U[0];
    T ux = U[1] * ir, uy = U[2] * ir;
    T p = (ph.gam - 1.0) * (U[3] - 0.5 * (U[1] * ux + U[2] * uy));
    T un = ux * n[0] + uy * n[1] - vn;
    return dsqrt(un * un + ph.lf_delta * ph.lf_delta) + dsqrt(ph.gam * p * ir);
}

// smoothed local Lax-Friedrichs: (H(UL)+H(UR))/2 - alpha (UR-UL)/2
template <class T>
__device__ __forceinline__ void flux_lf(const Phys& ph, const T UL[4], const T UR[4], const T n[2], const T& vn,
                                        T Fh[4])
{
    T HL[4], HR[4];
    flux_H(ph, UL, n, vn, HL);
    flux_H(ph, UR, n, vn, HR);
    T al = 0.5 * (wave_speed(ph, UL, n, vn) + wave_speed(ph, UR, n, vn));
#pragma unroll
    for (int m = 0; m < 4; ++m) Fh[m] = 0.5 * (HL[m] + HR[m]) - 0.5 * al * (UR[m] - UL[m]);
}

// ------------------------------------------------------------------ ALE geometry
// G[i][j] = dx_i/dX_j; cof G = g G^{-T}; Gi = G^{-1}
template <class T>
__device__ __forceinline__ void cof_inv(const T G[2][2], T cof[2][2], T Gi[2][2])
{
    T det = G[0][0] * G[1][1] - G[0][1] * G[1][0];
    T id = 1.0 / det;
    cof[0][0] = G[1][1];
    cof[0][1] = -G[1][0];
    cof[1][0] = -G[0][1];
    cof[1][1] = G[0][0];
    Gi[0][0] = G[1][1] * id;
    Gi[0][1] = -G[0][1] * id;
    Gi[1][0] = -G[1][0] * id;
    Gi[1][1] = G[0][0] * id;
}

// reference-domain volume flux F_X[m][D] at a point from the physical state U,
// its lifted X-gradient q[m][D], the map gradient G and the mesh velocity vG:
//   F_X = [F_inv(U) - F_vis(U, q G^{-1})] cof G - U (x) (cof G^T vG)
template <class T>
__device__ __forceinline__ void vol_flux(const Phys& ph, const T U[4], const T q[4][2], const T G[2][2],
                                         const T vG[2], T FX[4][2])
{
    T cof[2][2], Gi[2][2];
    cof_inv(G, cof, Gi);
    T dU[4][2], Fi[4][2], Fv[4][2];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        dU[m][0] = q[m][0] * Gi[0][0] + q[m][1] * Gi[1][0];
        dU[m][1] = q[m][0] * Gi[0][1] + q[m][1] * Gi[1][1];
    }
    flux_inv(ph, U, Fi);
    flux_vis(ph, U, dU, Fv, true);
    T w0 = cof[0][0] * vG[0] + cof[1][0] * vG[1];
    T w1 = cof[0][1] * vG[0] + cof[1][1] * vG[1];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        T a0 = Fi[m][0] - Fv[m][0], a1 = Fi[m][1] - Fv[m][1];
        FX[m][0] = a0 * cof[0][0] + a1 * cof[1][0] - U[m] * w0;
        FX[m][1] = a0 * cof[0][1] + a1 * cof[1][1] - U[m] * w1;
    }
}

// interior face flux Fhat . N^L (L side geometry G, vG; N outward of L in X):
//   j_f F_LF(UL, UR; n) - F_vis(UL, qL G^{-1}) (cof G N)
template <class T>
__device__ __forceinline__ void face_flux(const Phys& ph, const T UL[4], const T UR[4], const T qL[4][2],
                                          const T G[2][2], const T vG[2], const double N[2], T Fh[4])
{
    T cof[2][2], Gi[2][2];
    cof_inv(G, cof, Gi);
    T cn[2] = { cof[0][0] * N[0] + cof[0][1] * N[1], cof[1][0] * N[0] + cof[1][1] * N[1] };
    T jf = dsqrt(cn[0] * cn[0] + cn[1] * cn[1]);
    T ij = 1.0 / jf;
    T nn[2] = { cn[0] * ij, cn[1] * ij };
    T vn = vG[0] * nn[0] + vG[1] * nn[1];
    T Fi[4];
    flux_lf(ph, UL, UR, nn, vn, Fi);
    T dU[4][2], Fv[4][2];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        dU[m][0] = qL[m][0] * Gi[0][0] + qL[m][1] * Gi[1][0];
        dU[m][1] = qL[m][0] * Gi[0][1] + qL[m][1] * Gi[1][1];
    }
    flux_vis(ph, UL, dU, Fv, true);
#pragma unroll
    for (int m = 0; m < 4; ++m) Fh[m] = jf * Fi[m] - (Fv[m][0] * cn[0] + Fv[m][1] * cn[1]);
}

// boundary face flux Fhat . N_K.  wall: no-slip adiabatic moving wall --
// Lax-Friedrichs flux against the reflected state U_b (interior density and
// pressure, velocity 2 v_G - u: zero mass flux, average velocity = wall
// velocity), interior viscous stress without heat flux and an
// interior-penalty momentum term; otherwise far field against U_inf.
template <class T>
__device__ __forceinline__ void bnd_flux(const Phys& ph, bool wall, double hK, const T U[4], const T gU[4][2],
                                         const T G[2][2], const T vG[2], const double N[2], T Fh[4])
{
    T cof[2][2], Gi[2][2];
    cof_inv(G, cof, Gi);
    T cn[2] = { cof[0][0] * N[0] + cof[0][1] * N[1], cof[1][0] * N[0] + cof[1][1] * N[1] };
    T jf = dsqrt(cn[0] * cn[0] + cn[1] * cn[1]);
    T ij = 1.0 / jf;
    T nn[2] = { cn[0] * ij, cn[1] * ij };
    T vn = vG[0] * nn[0] + vG[1] * nn[1];
    T dU[4][2], Fv[4][2];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        dU[m][0] = gU[m][0] * Gi[0][0] + gU[m][1] * Gi[1][0];
        dU[m][1] = gU[m][0] * Gi[0][1] + gU[m][1] * Gi[1][1];
    }
    if (!wall) {
        T Ui[4] = { AD<T>::c(ph.Uinf[0]), AD<T>::c(ph.Uinf[1]), AD<T>::c(ph.Uinf[2]), AD<T>::c(ph.Uinf[3]) };
        T Fi[4];
        flux_lf(ph, U, Ui, nn, vn, Fi);
        flux_vis(ph, U, dU, Fv, true);
#pragma unroll
        for (int m = 0; m < 4; ++m) Fh[m] = jf * Fi[m] - (Fv[m][0] * cn[0] + Fv[m][1] * cn[1]);
    } else {
        T r = U[0];
        T ir = 1.0 / r;
        T ux = U[1] * ir, uy = U[2] * ir;
        // reflected state: interior density and pressure, velocity 2 v_G - u
        T bx = 2.0 * vG[0] - ux, by = 2.0 * vG[1] - uy;
        T Ub[4];
        Ub[0] = r;
        Ub[1] = r * bx;
        Ub[2] = r * by;
        Ub[3] = U[3] - 0.5 * r * (ux * ux + uy * uy) + 0.5 * r * (bx * bx + by * by);
        T H[4];
        flux_lf(ph, U, Ub, nn, vn, H);
        flux_vis(ph, U, dU, Fv, false);
        T tn0 = Fv[1][0] * nn[0] + Fv[1][1] * nn[1];
        T tn1 = Fv[2][0] * nn[0] + Fv[2][1] * nn[1];
        double pen = ph.muv * ph.wall_eta / hK;
        Fh[0] = jf * H[0];
        Fh[1] = jf * (H[1] - tn0 + pen * (U[1] - r * vG[0]));
        Fh[2] = jf * (H[2] - tn1 + pen * (U[2] - r * vG[1]));
        Fh[3] = jf * (H[3] - (vG[0] * tn0 + vG[1] * tn1));
    }
}

}  // namespace pa
