// HIP kernels of the periodic-adjoint library (gfx950, wave64).
//
// Discretisation (arXiv:1512.00616 Sec. 4 names nodal DG on triangles with
// the compact DG viscous treatment and an ALE map to a fixed reference
// domain; the details below are this library's reading):
//   r_{K,a} = int_K grad_X phi_a . F_X dX - oint_{dK} phi_a Fhat . N dS
//   U = U_X / gbar, q = grad_X U + sum of the liftings of the faces of which
//   K is the lower-index side; the lifting of face e lives on its lower-index
//   element L and satisfies int_L r_e : tau = -int_e (U^L - U^R) (x) N^L : tau.
//
// Element-per-workgroup kernels: a workgroup owns one element row K, reads
// the states of K and its three face neighbours, recomputes every shared
// face quantity in the lower-index element's orientation (bitwise identical
// from both sides, so the scheme stays exactly conservative) and writes only
// its own rows.  No atomics anywhere: all reductions have a fixed order.
#pragma once
#include "pa_device.hpp"

namespace pa {

template <int P>
struct Sz {
    static constexpr int NP = (P + 1) * (P + 2) / 2;
    static constexpr int NQ = (P + 2) * (P + 2);
    static constexpr int NF = P + 2;
    static constexpr int B = 4 * NP;
};

// reference-element tables (host-filled, device-resident)
template <int P>
struct Ref {
    static constexpr int NP = Sz<P>::NP, NQ = Sz<P>::NQ, NF = Sz<P>::NF;
    double phq[NQ][NP];          // basis at volume points
    double dphq[NQ][NP][2];      // reference gradient at volume points
    double wq[NQ];               // volume weights (sum 1/2)
    double phf[3][NF][NP];       // basis at face points, parameter s
    double dphf[3][NF][NP][2];
    double phr[3][NF][NP];       // basis at face points, parameter 1 - s
    double dphr[3][NF][NP][2];
    double wf[NF];               // face weights (sum 1)
    double mh[NP][NP];           // reference mass matrix
    double mhi[NP][NP];          // its inverse
};

struct DevMesh {
    int Ne;
    int wall_is_far;
    const int32_t* enb;     // [Ne][3] neighbour, -1 wall, -2 far field
    const int8_t* etw;      // [Ne][3] neighbour's local face
    const double* area;     // [Ne]
    const double* jit;      // [Ne][4] J_K^{-T}, row-major
    const double* xn;       // [Ne][NP][2] reference-domain node coordinates
    const double* wbl;      // [Ne][NP] mesh-motion blend weight at the nodes
    const double* elen;     // [Ne][3] edge length
    const double* enrm;     // [Ne][3][2] outward unit normal (reference domain)
};

// rigid heave/pitch values at one time (Sec. 4.1 eq. defmap): h, dh/dt,
// theta, dtheta/dt; T = Dual<3> carries their derivatives in (h0, theta0, phi)
template <class T>
struct Motion {
    T h, hd, th, thd;
};

template <class T>
__device__ __forceinline__ T load_g(const double* gb, const double* dgb, int64_t idx, int64_t nn);
template <>
__device__ __forceinline__ double load_g<double>(const double* gb, const double*, int64_t idx, int64_t)
{
    return gb[idx];
}
template <>
__device__ __forceinline__ Dual<3> load_g<Dual<3>>(const double* gb, const double* dgb, int64_t idx, int64_t nn)
{
    Dual<3> r;
    r.v = gb[idx];
    r.d[0] = dgb[idx];
    r.d[1] = dgb[nn + idx];
    r.d[2] = dgb[2 * nn + idx];
    return r;
}

// blended mesh motion at one node: x = X + w (Q X + v - X), v_G = w (theta' Q' X + v')
template <class T>
__device__ __forceinline__ void node_motion(double X, double Y, double w, const T& cs, const T& sn,
                                            const Motion<T>& mo, T x[2], T v[2])
{
    T qx = cs * X + sn * Y;
    T qy = -sn * X + cs * Y;
    x[0] = X + w * (qx - X);
    x[1] = Y + w * (qy + mo.h - Y);
    T dqx = -sn * X + cs * Y;
    T dqy = -cs * X - sn * Y;
    v[0] = w * (mo.thd * dqx);
    v[1] = w * (mo.thd * dqy + mo.hd);
}

// X-gradient of the basis at a point: jit * reference gradient
template <int NP>
__device__ __forceinline__ void grad_X(const double* jt, const double (*dph)[2], double (*gx)[2])
{
#pragma unroll
    for (int a = 0; a < NP; ++a) {
        gx[a][0] = jt[0] * dph[a][0] + jt[1] * dph[a][1];
        gx[a][1] = jt[2] * dph[a][0] + jt[3] * dph[a][1];
    }
}

// isoparametric geometry at a point from nodal x, v: G[i][j] = sum x_a,i dphi_a/dX_j
template <int NP, class T>
__device__ __forceinline__ void point_geom(const T (*x)[2], const T (*v)[2], const double* ph,
                                           const double (*gx)[2], T G[2][2], T vG[2])
{
    G[0][0] = G[0][1] = G[1][0] = G[1][1] = AD<T>::c(0.0);
    vG[0] = vG[1] = AD<T>::c(0.0);
#pragma unroll
    for (int a = 0; a < NP; ++a) {
        G[0][0] += x[a][0] * gx[a][0];
        G[0][1] += x[a][0] * gx[a][1];
        G[1][0] += x[a][1] * gx[a][0];
        G[1][1] += x[a][1] * gx[a][1];
        vG[0] += ph[a] * v[a][0];
        vG[1] += ph[a] * v[a][1];
    }
}

// physical state U = U_X / gbar and its X-gradient at a point
template <int NP, class T>
__device__ __forceinline__ void point_state(const T (*u)[4], const T* g, const double* ph, const double (*gx)[2],
                                            T U[4], T gU[4][2])
{
    T UX[4], dUX[4][2], gg = AD<T>::c(0.0), dg[2] = { AD<T>::c(0.0), AD<T>::c(0.0) };
#pragma unroll
    for (int m = 0; m < 4; ++m) UX[m] = dUX[m][0] = dUX[m][1] = AD<T>::c(0.0);
#pragma unroll
    for (int a = 0; a < NP; ++a) {
        gg += ph[a] * g[a];
        dg[0] += gx[a][0] * g[a];
        dg[1] += gx[a][1] * g[a];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            UX[m] += ph[a] * u[a][m];
            dUX[m][0] += gx[a][0] * u[a][m];
            dUX[m][1] += gx[a][1] * u[a][m];
        }
    }
    T ig = 1.0 / gg;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        U[m] = UX[m] * ig;
        if (gU) {
            gU[m][0] = (dUX[m][0] - U[m] * dg[0]) * ig;
            gU[m][1] = (dUX[m][1] - U[m] * dg[1]) * ig;
        }
    }
}

// ------------------------------------------------------------------ residual
// One 64-lane workgroup per element.  T = double gives r(u); T = Dual<3>
// carries d/dmu through the mesh motion and gbar (out[k*Nu + .] = dr/dmu_k,
// and the value part is not written).
template <int P, class T>
__global__ void __launch_bounds__(64) k_residual(DevMesh M, const Ref<P>* __restrict__ R, Phys ph, Motion<T> mo,
                                                 const double* __restrict__ u, const double* __restrict__ gb,
                                                 const double* __restrict__ dgb, double* __restrict__ out, int64_t Nu)
{
    constexpr int NP = Sz<P>::NP, NQ = Sz<P>::NQ, NF = Sz<P>::NF, B = Sz<P>::B;
    const int K = blockIdx.x, tid = threadIdx.x;
    const int64_t nn = (int64_t)M.Ne * NP;
    __shared__ T sU[4][NP][4];
    __shared__ T sg[4][NP];
    __shared__ T sx[4][NP][2], sv[4][NP][2];
    __shared__ T sUL[3][NF][4], sdel[3][NF][4], sgUL[3][NF][4][2];
    __shared__ T slift[3][NP][4];
    __shared__ T sFh[3][NF][4];
    __shared__ T sFX[NQ][4][2];
    int nb[3], tw[3];
#pragma unroll
    for (int f = 0; f < 3; ++f) { nb[f] = M.enb[3 * K + f]; tw[f] = M.etw[3 * K + f]; }
    T cs, sn;
    dsincos(mo.th, &sn, &cs);
    // load K (slot 0) and its neighbours (slots 1..3)
    for (int idx = tid; idx < 4 * NP; idx += blockDim.x) {
        int e = idx / NP, a = idx % NP;
        int E = e == 0 ? K : nb[e - 1];
        if (E < 0) continue;
        int64_t na = (int64_t)E * NP + a;
#pragma unroll
        for (int m = 0; m < 4; ++m) sU[e][a][m] = AD<T>::c(u[na * 4 + m]);
        sg[e][a] = load_g<T>(gb, dgb, na, nn);
        T x[2], v[2];
        node_motion(M.xn[2 * na], M.xn[2 * na + 1], M.wbl[na], cs, sn, mo, x, v);
        sx[e][a][0] = x[0]; sx[e][a][1] = x[1];
        sv[e][a][0] = v[0]; sv[e][a][1] = v[1];
    }
    __syncthreads();
    // phase 1: face traces (lower-index element's orientation)
    if (tid < 3 * NF) {
        int f = tid / NF, j = tid % NF;
        double gx[NP][2];
        if (nb[f] >= 0) {
            bool KL = K < nb[f];
            int Ls = KL ? 0 : 1 + f, Rs = KL ? 1 + f : 0;
            int L = KL ? K : nb[f], Rr = KL ? nb[f] : K;
            int fL = KL ? f : tw[f], fR = KL ? tw[f] : f;
            T UL[4], gUL[4][2], UR[4];
            grad_X<NP>(M.jit + 4 * L, R->dphf[fL][j], gx);
            point_state<NP, T>(sU[Ls], sg[Ls], R->phf[fL][j], gx, UL, gUL);
            grad_X<NP>(M.jit + 4 * Rr, R->dphr[fR][j], gx);
            point_state<NP, T>(sU[Rs], sg[Rs], R->phr[fR][j], gx, UR, nullptr);
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                sUL[f][j][m] = UL[m];
                sdel[f][j][m] = UL[m] - UR[m];
                sgUL[f][j][m][0] = gUL[m][0];
                sgUL[f][j][m][1] = gUL[m][1];
            }
        } else {
            T U[4], gU[4][2];
            grad_X<NP>(M.jit + 4 * K, R->dphf[f][j], gx);
            point_state<NP, T>(sU[0], sg[0], R->phf[f][j], gx, U, gU);
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                sUL[f][j][m] = U[m];
                sgUL[f][j][m][0] = gU[m][0];
                sgUL[f][j][m][1] = gU[m][1];
            }
        }
    }
    __syncthreads();
    // phase 2: lifting coefficients (scalar part; times N^L_D when used)
    for (int t = tid; t < 3 * NP * 4; t += blockDim.x) {
        int f = t / (NP * 4), c = (t / 4) % NP, m = t % 4;
        if (nb[f] < 0) continue;
        bool KL = K < nb[f];
        int L = KL ? K : nb[f], fL = KL ? f : tw[f];
        double s = -M.elen[3 * K + f] / (2.0 * M.area[L]);
        T acc = AD<T>::c(0.0);
#pragma unroll
        for (int cp = 0; cp < NP; ++cp) {
            T t2 = AD<T>::c(0.0);
#pragma unroll
            for (int j = 0; j < NF; ++j) t2 += (R->wf[j] * R->phf[fL][j][cp]) * sdel[f][j][m];
            acc += R->mhi[c][cp] * t2;
        }
        slift[f][c][m] = s * acc;
    }
    __syncthreads();
    // phase 3: face fluxes
    if (tid < 3 * NF) {
        int f = tid / NF, j = tid % NF;
        double gx[NP][2];
        T G[2][2], vG[2], Fh[4];
        if (nb[f] >= 0) {
            bool KL = K < nb[f];
            int Ls = KL ? 0 : 1 + f, L = KL ? K : nb[f], fL = KL ? f : tw[f];
            const double* N = M.enrm + 2 * (3 * L + fL);
            grad_X<NP>(M.jit + 4 * L, R->dphf[fL][j], gx);
            point_geom<NP, T>(sx[Ls], sv[Ls], R->phf[fL][j], gx, G, vG);
            T q[4][2];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                T l = AD<T>::c(0.0);
#pragma unroll
                for (int c = 0; c < NP; ++c) l += R->phf[fL][j][c] * slift[f][c][m];
                q[m][0] = sgUL[f][j][m][0] + l * N[0];
                q[m][1] = sgUL[f][j][m][1] + l * N[1];
            }
            T UR[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) UR[m] = sUL[f][j][m] - sdel[f][j][m];
            face_flux(ph, sUL[f][j], UR, q, G, vG, N, Fh);
        } else {
            const double* N = M.enrm + 2 * (3 * K + f);
            grad_X<NP>(M.jit + 4 * K, R->dphf[f][j], gx);
            point_geom<NP, T>(sx[0], sv[0], R->phf[f][j], gx, G, vG);
            bool wall = (nb[f] == -1) && !M.wall_is_far;
            double hK = 2.0 * M.area[K] / M.elen[3 * K + f];
            bnd_flux(ph, wall, hK, sUL[f][j], sgUL[f][j], G, vG, N, Fh);
        }
#pragma unroll
        for (int m = 0; m < 4; ++m) sFh[f][j][m] = Fh[m];
    }
    // phase 4: volume fluxes
    for (int q = tid; q < NQ; q += blockDim.x) {
        double gx[NP][2];
        grad_X<NP>(M.jit + 4 * K, R->dphq[q], gx);
        T U[4], gU[4][2], G[2][2], vG[2], FX[4][2];
        point_state<NP, T>(sU[0], sg[0], R->phq[q], gx, U, gU);
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            if (!(nb[f] > K)) continue;
            const double* N = M.enrm + 2 * (3 * K + f);
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                T l = AD<T>::c(0.0);
#pragma unroll
                for (int c = 0; c < NP; ++c) l += R->phq[q][c] * slift[f][c][m];
                gU[m][0] += l * N[0];
                gU[m][1] += l * N[1];
            }
        }
        point_geom<NP, T>(sx[0], sv[0], R->phq[q], gx, G, vG);
        vol_flux(ph, U, gU, G, vG, FX);
#pragma unroll
        for (int m = 0; m < 4; ++m) { sFX[q][m][0] = FX[m][0]; sFX[q][m][1] = FX[m][1]; }
    }
    __syncthreads();
    // phase 5: test-function integrals
    if (tid < B) {
        int a = tid / 4, m = tid % 4;
        const double* jt = M.jit + 4 * K;
        T acc = AD<T>::c(0.0);
        for (int q = 0; q < NQ; ++q) {
            double g0 = jt[0] * R->dphq[q][a][0] + jt[1] * R->dphq[q][a][1];
            double g1 = jt[2] * R->dphq[q][a][0] + jt[3] * R->dphq[q][a][1];
            acc += R->wq[q] * (g0 * sFX[q][m][0] + g1 * sFX[q][m][1]);
        }
        acc = (2.0 * M.area[K]) * acc;
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            double sgn = (nb[f] >= 0 && nb[f] < K) ? -1.0 : 1.0;
            T s = AD<T>::c(0.0);
#pragma unroll
            for (int j = 0; j < NF; ++j) {
                double pa = (nb[f] >= 0 && nb[f] < K) ? R->phr[f][j][a] : R->phf[f][j][a];
                s += (R->wf[j] * pa) * sFh[f][j][m];
            }
            acc -= (sgn * M.elen[3 * K + f]) * s;
        }
        int64_t idx = (int64_t)K * B + tid;
        if constexpr (sizeof(T) == sizeof(double)) {
            out[idx] = AD<T>::val(acc);
        } else {
            const double* dd = reinterpret_cast<const double*>(&acc) + 1;
            out[idx] = dd[0];
            out[Nu + idx] = dd[1];
            out[2 * Nu + idx] = dd[2];
        }
    }
}

// ------------------------------------------------------------------ Jacobian
// dr/du of the element row K as four b x b blocks (diagonal, then the
// neighbours across faces 0, 1, 2), from exact pointwise flux Jacobians
// (dual numbers) contracted with the basis/trace/lifting operators.
template <int P>
struct JacSmem {
    static constexpr int NP = Sz<P>::NP, NQ = Sz<P>::NQ, NF = Sz<P>::NF;
    double U[4][NP][4];
    double g[4][NP];
    double x[4][NP][2], v[4][NP][2];
    // face data, point index j in the lower-index side's orientation
    double UL[3][NF][4], UR[3][NF][4], gUL[3][NF][4][2];
    double gL[3][NF], gR[3][NF];        // 1 / gbar at the face points of either side
    double GL[3][NF][2][2], vGL[3][NF][2];
    double lift[3][NP][4];
    double LamL[3][NP][NP], LamR[3][NP][NP];
    double BuL[3][NF][NP], BuR[3][NF][NP];   // phi_b / gbar on either side
    double PsiL[3][NF][NP][2];               // d q^L / d U_X^L (per component)
    double LRf[3][NF][NP];                   // sum_c phi^L_c Lam^R[c][b]
    double E[3][NF][4][16];                  // face pointwise Jacobians
    // volume data
    double Uq[NQ][4], qq[NQ][4][2], Gq[NQ][2][2], vGq[NQ][2];
    double Buq[NQ][NP], Psi0[NQ][NP][2], LRv[3][NQ][NP];
    double gphq[NQ][NP][2];
    double D[NQ][4][2][12];                  // volume pointwise Jacobians
};

typedef double mf_d4 __attribute__((ext_vector_type(4)));   // FP64 MFMA accumulator

template <int P>
__global__ void __launch_bounds__(320) k_jacobian(DevMesh M, const Ref<P>* __restrict__ R, Phys ph, Motion<double> mo,
                                                  const double* __restrict__ u, const double* __restrict__ gb,
                                                  double* __restrict__ J)
{
    constexpr int NP = Sz<P>::NP, NQ = Sz<P>::NQ, NF = Sz<P>::NF, B = Sz<P>::B;
    using D1 = Dual<1>;
    extern __shared__ double smem_raw[];
    JacSmem<P>& S = *reinterpret_cast<JacSmem<P>*>(smem_raw);
    const int K = blockIdx.x, tid = threadIdx.x, nth = blockDim.x;
    int nb[3], tw[3];
#pragma unroll
    for (int f = 0; f < 3; ++f) { nb[f] = M.enb[3 * K + f]; tw[f] = M.etw[3 * K + f]; }
    double cs = cos(mo.th), sn = sin(mo.th);
    for (int idx = tid; idx < 4 * NP; idx += nth) {
        int e = idx / NP, a = idx % NP;
        int E = e == 0 ? K : nb[e - 1];
        if (E < 0) continue;
        int64_t na = (int64_t)E * NP + a;
#pragma unroll
        for (int m = 0; m < 4; ++m) S.U[e][a][m] = u[na * 4 + m];
        S.g[e][a] = gb[na];
        double x[2], v[2];
        node_motion(M.xn[2 * na], M.xn[2 * na + 1], M.wbl[na], cs, sn, mo, x, v);
        S.x[e][a][0] = x[0]; S.x[e][a][1] = x[1];
        S.v[e][a][0] = v[0]; S.v[e][a][1] = v[1];
    }
    const double* jtK = M.jit + 4 * K;
    for (int t = tid; t < NQ * NP; t += nth) {
        int q = t / NP, a = t % NP;
        S.gphq[q][a][0] = jtK[0] * R->dphq[q][a][0] + jtK[1] * R->dphq[q][a][1];
        S.gphq[q][a][1] = jtK[2] * R->dphq[q][a][0] + jtK[3] * R->dphq[q][a][1];
    }
    __syncthreads();
    // phase 1: face traces and trace operators
    for (int t = tid; t < 3 * NF; t += nth) {
        int f = t / NF, j = t % NF;
        double gx[NP][2];
        double G[2][2], vG[2];
        if (nb[f] >= 0) {
            bool KL = K < nb[f];
            int Ls = KL ? 0 : 1 + f, Rs = KL ? 1 + f : 0;
            int L = KL ? K : nb[f], Rr = KL ? nb[f] : K;
            int fL = KL ? f : tw[f], fR = KL ? tw[f] : f;
            double UL[4], gUL[4][2], UR[4];
            grad_X<NP>(M.jit + 4 * L, R->dphf[fL][j], gx);
            point_state<NP, double>(S.U[Ls], S.g[Ls], R->phf[fL][j], gx, UL, gUL);
            point_geom<NP, double>(S.x[Ls], S.v[Ls], R->phf[fL][j], gx, G, vG);
            double gl = 0, dgl[2] = { 0, 0 };
            for (int a = 0; a < NP; ++a) { gl += R->phf[fL][j][a] * S.g[Ls][a]; dgl[0] += gx[a][0] * S.g[Ls][a]; dgl[1] += gx[a][1] * S.g[Ls][a]; }
            const double igl = 1.0 / gl, igl2 = igl * igl;   // one division per point
            for (int b = 0; b < NP; ++b) {
                S.BuL[f][j][b] = R->phf[fL][j][b] * igl;
                S.PsiL[f][j][b][0] = gx[b][0] * igl - R->phf[fL][j][b] * dgl[0] * igl2;
                S.PsiL[f][j][b][1] = gx[b][1] * igl - R->phf[fL][j][b] * dgl[1] * igl2;
            }
            grad_X<NP>(M.jit + 4 * Rr, R->dphr[fR][j], gx);
            point_state<NP, double>(S.U[Rs], S.g[Rs], R->phr[fR][j], gx, UR, nullptr);
            double gr = 0;
            for (int a = 0; a < NP; ++a) gr += R->phr[fR][j][a] * S.g[Rs][a];
            const double igr = 1.0 / gr;
            for (int b = 0; b < NP; ++b) S.BuR[f][j][b] = R->phr[fR][j][b] * igr;
            S.gL[f][j] = igl;   // the lifting operators use the reciprocals
            S.gR[f][j] = igr;
            for (int m = 0; m < 4; ++m) {
                S.UL[f][j][m] = UL[m];
                S.UR[f][j][m] = UR[m];
                S.gUL[f][j][m][0] = gUL[m][0];
                S.gUL[f][j][m][1] = gUL[m][1];
            }
        } else {
            double U[4], gU[4][2];
            grad_X<NP>(jtK, R->dphf[f][j], gx);
            point_state<NP, double>(S.U[0], S.g[0], R->phf[f][j], gx, U, gU);
            point_geom<NP, double>(S.x[0], S.v[0], R->phf[f][j], gx, G, vG);
            double gl = 0, dgl[2] = { 0, 0 };
            for (int a = 0; a < NP; ++a) { gl += R->phf[f][j][a] * S.g[0][a]; dgl[0] += gx[a][0] * S.g[0][a]; dgl[1] += gx[a][1] * S.g[0][a]; }
            const double igl = 1.0 / gl, igl2 = igl * igl;
            for (int b = 0; b < NP; ++b) {
                S.BuL[f][j][b] = R->phf[f][j][b] * igl;
                S.PsiL[f][j][b][0] = gx[b][0] * igl - R->phf[f][j][b] * dgl[0] * igl2;
                S.PsiL[f][j][b][1] = gx[b][1] * igl - R->phf[f][j][b] * dgl[1] * igl2;
            }
            for (int m = 0; m < 4; ++m) {
                S.UL[f][j][m] = U[m];
                S.gUL[f][j][m][0] = gU[m][0];
                S.gUL[f][j][m][1] = gU[m][1];
            }
        }
        for (int a = 0; a < 2; ++a) {
            S.GL[f][j][a][0] = G[a][0];
            S.GL[f][j][a][1] = G[a][1];
            S.vGL[f][j][a] = vG[a];
        }
    }
    // volume point values
    for (int q = tid; q < NQ; q += nth) {
        double G[2][2], vG[2], U[4], gU[4][2];
        point_state<NP, double>(S.U[0], S.g[0], R->phq[q], S.gphq[q], U, gU);
        point_geom<NP, double>(S.x[0], S.v[0], R->phq[q], S.gphq[q], G, vG);
        double gg = 0, dg[2] = { 0, 0 };
        for (int a = 0; a < NP; ++a) { gg += R->phq[q][a] * S.g[0][a]; dg[0] += S.gphq[q][a][0] * S.g[0][a]; dg[1] += S.gphq[q][a][1] * S.g[0][a]; }
        const double igg = 1.0 / gg, igg2 = igg * igg;
        for (int b = 0; b < NP; ++b) {
            S.Buq[q][b] = R->phq[q][b] * igg;
            S.Psi0[q][b][0] = S.gphq[q][b][0] * igg - R->phq[q][b] * dg[0] * igg2;
            S.Psi0[q][b][1] = S.gphq[q][b][1] * igg - R->phq[q][b] * dg[1] * igg2;
        }
        for (int m = 0; m < 4; ++m) { S.Uq[q][m] = U[m]; S.qq[q][m][0] = gU[m][0]; S.qq[q][m][1] = gU[m][1]; }
        for (int a = 0; a < 2; ++a) { S.Gq[q][a][0] = G[a][0]; S.Gq[q][a][1] = G[a][1]; S.vGq[q][a] = vG[a]; }
    }
    __syncthreads();
    // phase 2: lifting values and lifting operators Lam^L, Lam^R
    for (int t = tid; t < 3 * NP * 4; t += nth) {
        int f = t / (NP * 4), c = (t / 4) % NP, m = t % 4;
        if (nb[f] < 0) continue;
        bool KL = K < nb[f];
        int L = KL ? K : nb[f], fL = KL ? f : tw[f];
        double s = -M.elen[3 * K + f] / (2.0 * M.area[L]);
        double acc = 0;
        for (int cp = 0; cp < NP; ++cp) {
            double t2 = 0;
            for (int j = 0; j < NF; ++j) t2 += R->wf[j] * R->phf[fL][j][cp] * (S.UL[f][j][m] - S.UR[f][j][m]);
            acc += R->mhi[c][cp] * t2;
        }
        S.lift[f][c][m] = s * acc;
    }
    // lifting operators Lam = +-s Mhat^{-1} T with T[cp][b] = sum_j wf_j
    // phi_cp(j) phi_b(j) / gbar(j) on either side: T first (one face point sum
    // per entry), then the product with the inverse reference mass matrix.
    // T lives in the element-data arrays, which no later phase reads.
    {
        double* Tt = &S.U[0][0][0];   // 3 NP^2 doubles (U, g, x, v are contiguous and dead here)
        static_assert(sizeof(S.U) + sizeof(S.g) + sizeof(S.x) + sizeof(S.v) >= 3 * NP * NP * sizeof(double),
                      "room for the lifting sums");
        for (int side = 0; side < 2; ++side) {
            for (int t = tid; t < 3 * NP * NP; t += nth) {
                const int f = t / (NP * NP), cp = (t / NP) % NP, b = t % NP;
                if (nb[f] < 0) continue;
                const bool KL = K < nb[f];
                const int fL = KL ? f : tw[f], fR = KL ? tw[f] : f;
                double acc = 0.0;
                for (int j = 0; j < NF; ++j) {
                    const double w = R->wf[j] * R->phf[fL][j][cp];
                    acc += side == 0 ? w * R->phf[fL][j][b] * S.gL[f][j] : w * R->phr[fR][j][b] * S.gR[f][j];
                }
                Tt[t] = acc;
            }
            __syncthreads();
            for (int t = tid; t < 3 * NP * NP; t += nth) {
                const int f = t / (NP * NP), c = (t / NP) % NP, b = t % NP;
                if (nb[f] < 0) continue;
                const bool KL = K < nb[f];
                const int L = KL ? K : nb[f];
                const double s = -M.elen[3 * K + f] / (2.0 * M.area[L]);
                double a = 0.0;
                for (int cp = 0; cp < NP; ++cp) a += R->mhi[c][cp] * Tt[(f * NP + cp) * NP + b];
                if (side == 0) S.LamL[f][c][b] = s * a;
                else S.LamR[f][c][b] = -s * a;
            }
            __syncthreads();
        }
    }
    __syncthreads();
    // lifting contributions to the trace and volume gradient operators
    for (int t = tid; t < 3 * NF * NP; t += nth) {
        int f = t / (NF * NP), j = (t / NP) % NF, b = t % NP;
        if (nb[f] < 0) continue;
        bool KL = K < nb[f];
        int L = KL ? K : nb[f], fL = KL ? f : tw[f];
        const double* N = M.enrm + 2 * (3 * L + fL);
        double sl = 0, sr = 0;
        for (int c = 0; c < NP; ++c) {
            sl += R->phf[fL][j][c] * S.LamL[f][c][b];
            sr += R->phf[fL][j][c] * S.LamR[f][c][b];
        }
        S.PsiL[f][j][b][0] += sl * N[0];
        S.PsiL[f][j][b][1] += sl * N[1];
        S.LRf[f][j][b] = sr;
    }
    for (int t = tid; t < NQ * NP; t += nth) {
        int q = t / NP, b = t % NP;
        for (int f = 0; f < 3; ++f) {
            if (!(nb[f] > K)) continue;
            const double* N = M.enrm + 2 * (3 * K + f);
            double sl = 0, sr = 0;
            for (int c = 0; c < NP; ++c) {
                sl += R->phq[q][c] * S.LamL[f][c][b];
                sr += R->phq[q][c] * S.LamR[f][c][b];
            }
            S.Psi0[q][b][0] += sl * N[0];
            S.Psi0[q][b][1] += sl * N[1];
            S.LRv[f][q][b] = sr;
        }
    }
    // lifted gradients at volume and face points (values)
    for (int t = tid; t < NQ * 4; t += nth) {
        int q = t / 4, m = t % 4;
        for (int f = 0; f < 3; ++f) {
            if (!(nb[f] > K)) continue;
            const double* N = M.enrm + 2 * (3 * K + f);
            double l = 0;
            for (int c = 0; c < NP; ++c) l += R->phq[q][c] * S.lift[f][c][m];
            S.qq[q][m][0] += l * N[0];
            S.qq[q][m][1] += l * N[1];
        }
    }
    for (int t = tid; t < 3 * NF * 4; t += nth) {
        int f = t / (NF * 4), j = (t / 4) % NF, m = t % 4;
        if (nb[f] < 0) continue;
        bool KL = K < nb[f];
        int L = KL ? K : nb[f], fL = KL ? f : tw[f];
        const double* N = M.enrm + 2 * (3 * L + fL);
        double l = 0;
        for (int c = 0; c < NP; ++c) l += R->phf[fL][j][c] * S.lift[f][c][m];
        S.gUL[f][j][m][0] += l * N[0];
        S.gUL[f][j][m][1] += l * N[1];
    }
    __syncthreads();
    // test-side (A) values of the contraction, formed once: the volume ones
    // in place of the basis gradients (w2K wq[q] grad phi_a(q), which only the
    // contraction reads from here on), the face ones in the dead lifting-
    // operator storage (-sign |e| wf[j] phi_a at the face point, from K's
    // side of the face)
    {
        const double w2K = 2.0 * M.area[K];
        for (int t = tid; t < NQ * NP; t += nth) {
            const int q = t / NP, a = t % NP;
            const double wq = w2K * R->wq[q];
            S.gphq[q][a][0] *= wq;
            S.gphq[q][a][1] *= wq;
        }
        double* Af = &S.LamL[0][0][0];   // [3][NF][NP]
        for (int t = tid; t < 3 * NF * NP; t += nth) {
            const int ff = t / (NF * NP), j = (t / NP) % NF, a = t % NP;
            const double len = M.elen[3 * K + ff];
            double v;
            if (nb[ff] >= 0) {
                const bool KL = K < nb[ff];
                const double sg = (KL ? 1.0 : -1.0) * len;
                v = -sg * R->wf[j] * (KL ? R->phf[ff][j][a] : R->phr[ff][j][a]);
            } else {
                v = -len * R->wf[j] * R->phf[ff][j][a];
            }
            Af[t] = v;
        }
    }
    // phase 3: pointwise Jacobians (one dual direction per thread)
    for (int t = tid; t < NQ * 12; t += nth) {
        int q = t / 12, sd = t % 12;
        D1 U[4], qv[4][2], G[2][2], vG[2], FX[4][2];
        for (int m = 0; m < 4; ++m) {
            U[m] = AD<D1>::c(S.Uq[q][m]);
            qv[m][0] = AD<D1>::c(S.qq[q][m][0]);
            qv[m][1] = AD<D1>::c(S.qq[q][m][1]);
        }
        if (sd < 4) U[sd].d[0] = 1.0;
        else qv[(sd - 4) >> 1][(sd - 4) & 1].d[0] = 1.0;
        for (int a = 0; a < 2; ++a) {
            G[a][0] = AD<D1>::c(S.Gq[q][a][0]);
            G[a][1] = AD<D1>::c(S.Gq[q][a][1]);
            vG[a] = AD<D1>::c(S.vGq[q][a]);
        }
        vol_flux(ph, U, qv, G, vG, FX);
        for (int m = 0; m < 4; ++m) {
            S.D[q][m][0][sd] = FX[m][0].d[0];
            S.D[q][m][1][sd] = FX[m][1].d[0];
        }
    }
    for (int t = tid; t < 3 * NF * 16; t += nth) {
        int f = t / (NF * 16), j = (t / 16) % NF, sd = t % 16;
        D1 G[2][2], vG[2], Fh[4];
        for (int a = 0; a < 2; ++a) {
            G[a][0] = AD<D1>::c(S.GL[f][j][a][0]);
            G[a][1] = AD<D1>::c(S.GL[f][j][a][1]);
            vG[a] = AD<D1>::c(S.vGL[f][j][a]);
        }
        if (nb[f] >= 0) {
            bool KL = K < nb[f];
            int L = KL ? K : nb[f], fL = KL ? f : tw[f];
            const double* N = M.enrm + 2 * (3 * L + fL);
            D1 UL[4], UR[4], q[4][2];
            for (int m = 0; m < 4; ++m) {
                UL[m] = AD<D1>::c(S.UL[f][j][m]);
                UR[m] = AD<D1>::c(S.UR[f][j][m]);
                q[m][0] = AD<D1>::c(S.gUL[f][j][m][0]);
                q[m][1] = AD<D1>::c(S.gUL[f][j][m][1]);
            }
            if (sd < 4) UL[sd].d[0] = 1.0;
            else if (sd < 8) UR[sd - 4].d[0] = 1.0;
            else q[(sd - 8) >> 1][(sd - 8) & 1].d[0] = 1.0;
            face_flux(ph, UL, UR, q, G, vG, N, Fh);
        } else {
            if (sd >= 12) { for (int m = 0; m < 4; ++m) S.E[f][j][m][sd] = 0.0; continue; }
            const double* N = M.enrm + 2 * (3 * K + f);
            D1 U[4], q[4][2];
            for (int m = 0; m < 4; ++m) {
                U[m] = AD<D1>::c(S.UL[f][j][m]);
                q[m][0] = AD<D1>::c(S.gUL[f][j][m][0]);
                q[m][1] = AD<D1>::c(S.gUL[f][j][m][1]);
            }
            if (sd < 4) U[sd].d[0] = 1.0;
            else q[(sd - 4) >> 1][(sd - 4) & 1].d[0] = 1.0;
            bool wall = (nb[f] == -1) && !M.wall_is_far;
            double hK = 2.0 * M.area[K] / M.elen[3 * K + f];
            bnd_flux(ph, wall, hK, U, q, G, vG, N, Fh);
        }
        for (int m = 0; m < 4; ++m) S.E[f][j][m][sd] = Fh[m].d[0];
    }
    __syncthreads();
    // phase 4: contract into the four blocks of row K on the FP64 matrix
    // cores.  Every term of a block has the form
    //   J[a][(m,n,b)] = sum_p  L_p[a] * Z_p[(m,n,b)]
    // over pseudo-points p (volume point and gradient direction, or face
    // point): L_p holds the test side (weighted basis or gradient values),
    // Z_p a short sum of pointwise-Jacobian entries times trial-side
    // operators.  That is a product (NP x P) x (P x 16 NP): M = test
    // function a (padded to 16), N = column (m, b, n) in NP tiles of 16,
    // K = pseudo-points in steps of 4 (v_mfma_f64_16x16x4).  Each lane
    // forms its A value L_p[a] and its B value Z_p[col] on the fly from LDS.
    // Lane layout: A[i][k] from lane i + 16 k, B[k][j] from lane j + 16 k,
    // result (lane / 16 + 4 r, lane % 16) in register r.  Tasks: (block s,
    // column tile), spread over the waves.
    {
        const double* Af = &S.LamL[0][0][0];   // face A values, [3][NF][NP]
        const int wave = tid >> 6, nwaves = nth >> 6, lane = tid & 63;
        const int li = lane & 15, lk = lane >> 4;
        // a task is two column tiles of one block: they share the test-side
        // A values, and their two accumulator chains run side by side
        constexpr int NT2 = (NP + 1) / 2;
        for (int task = wave; task < 4 * NT2; task += nwaves) {
            const int s_ = task / NT2, tile0 = 2 * (task % NT2);
            const bool two = tile0 + 1 < NP;
            // B column cc of this lane = (row variable m, trial function b,
            // column variable n) with n fastest: consecutive lanes hold
            // consecutive columns b * 4 + n of the block row, so the stores
            // of a result row are contiguous
            int bb[2], nn[2], mm[2];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const int cc = (tile0 + (two ? t : 0)) * 16 + li;
                nn[t] = cc & 3;
                bb[t] = (cc >> 2) % NP;
                mm[t] = (cc >> 2) / NP;
            }
            mf_d4 acc0 = { 0.0, 0.0, 0.0, 0.0 }, acc1 = { 0.0, 0.0, 0.0, 0.0 };
            const int f = s_ - 1;
            const bool volume = s_ == 0 || (nb[f] >= 0 && K < nb[f]);
            if (volume) {
                const double* NK = s_ == 0 ? nullptr : M.enrm + 2 * (3 * K + f);
#pragma unroll
                for (int ks = 0; ks < (2 * NQ + 3) / 4; ++ks) {
                    const int kk = 4 * ks + lk;
                    double av = 0.0, bv[2] = { 0.0, 0.0 };
                    if (kk < 2 * NQ) {
                        const int q = kk >> 1, d = kk & 1;
                        if (li < NP) av = S.gphq[q][li][d];
#pragma unroll
                        for (int t = 0; t < 2; ++t) {
                            const int m = mm[t], n = nn[t], b = bb[t];
                            if (s_ == 0)
                                bv[t] = S.D[q][m][d][n] * S.Buq[q][b] + S.D[q][m][d][4 + 2 * n] * S.Psi0[q][b][0] +
                                        S.D[q][m][d][5 + 2 * n] * S.Psi0[q][b][1];
                            else
                                bv[t] = (S.D[q][m][d][4 + 2 * n] * NK[0] + S.D[q][m][d][5 + 2 * n] * NK[1]) *
                                        S.LRv[f][q][b];
                        }
                    }
                    acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv[0], acc0, 0, 0, 0);
                    acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv[1], acc1, 0, 0, 0);
                }
            }
            // face terms: the three faces of K (diagonal block) or face f
            const int npts = s_ == 0 ? 3 * NF : (nb[f] >= 0 ? NF : 0);
            for (int ks = 0; ks < (npts + 3) / 4; ++ks) {
                const int kk = 4 * ks + lk;
                double av = 0.0, bv[2] = { 0.0, 0.0 };
                if (kk < npts) {
                    const int ff = s_ == 0 ? kk / NF : f, j = s_ == 0 ? kk % NF : kk;
                    if (nb[ff] >= 0) {
                        const bool KL = K < nb[ff];
                        const int L = KL ? K : nb[ff], fL = KL ? ff : tw[ff];
                        const double* N = M.enrm + 2 * (3 * L + fL);
                        // the diagonal block takes K's own trace, a neighbour block the other side's
                        const bool own = (s_ == 0) == KL;
#pragma unroll
                        for (int t = 0; t < 2; ++t) {
                            const int m = mm[t], n = nn[t], b = bb[t];
                            if (own)
                                bv[t] = S.E[ff][j][m][n] * S.BuL[ff][j][b] +
                                        S.E[ff][j][m][8 + 2 * n] * S.PsiL[ff][j][b][0] +
                                        S.E[ff][j][m][9 + 2 * n] * S.PsiL[ff][j][b][1];
                            else
                                bv[t] = S.E[ff][j][m][4 + n] * S.BuR[ff][j][b] +
                                        (S.E[ff][j][m][8 + 2 * n] * N[0] + S.E[ff][j][m][9 + 2 * n] * N[1]) *
                                            S.LRf[ff][j][b];
                        }
                        if (li < NP) av = Af[(ff * NF + j) * NP + li];
                    } else {
#pragma unroll
                        for (int t = 0; t < 2; ++t) {
                            const int m = mm[t], n = nn[t], b = bb[t];
                            bv[t] = S.E[ff][j][m][n] * S.BuL[ff][j][b] + S.E[ff][j][m][4 + 2 * n] * S.PsiL[ff][j][b][0] +
                                    S.E[ff][j][m][5 + 2 * n] * S.PsiL[ff][j][b][1];
                        }
                        if (li < NP) av = Af[(ff * NF + j) * NP + li];
                    }
                }
                acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv[0], acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv[1], acc1, 0, 0, 0);
            }
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                if (t == 1 && !two) break;
                double* Jb = J + (int64_t)K * 4 * B * B + (int64_t)s_ * B * B + mm[t] * B + bb[t] * 4 + nn[t];
                const mf_d4& ac = t == 0 ? acc0 : acc1;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int a = lk + 4 * r;
                    if (a < NP) Jb[a * 4 * B] = ac[r];
                }
            }
        }
    }
}

// ------------------------------------------------------------------ GCL field
// r_g,a = -int grad phi_a . (cof G^T v_G) + oint phi_a v_G . (cof G N)
template <int P, class T>
__global__ void __launch_bounds__(64) k_gcl_rhs(DevMesh M, const Ref<P>* __restrict__ R, Motion<T> mo,
                                                double* __restrict__ out, int64_t nn)
{
    constexpr int NP = Sz<P>::NP, NQ = Sz<P>::NQ, NF = Sz<P>::NF;
    const int K = blockIdx.x, tid = threadIdx.x;
    __shared__ T sx[4][NP][2], sv[4][NP][2];
    __shared__ T sw[NQ][2];
    __shared__ T sfl[3][NF];
    int nb[3], tw[3];
    for (int f = 0; f < 3; ++f) { nb[f] = M.enb[3 * K + f]; tw[f] = M.etw[3 * K + f]; }
    T cs, sn;
    dsincos(mo.th, &sn, &cs);
    for (int idx = tid; idx < 4 * NP; idx += blockDim.x) {
        int e = idx / NP, a = idx % NP;
        int E = e == 0 ? K : nb[e - 1];
        if (E < 0) continue;
        int64_t na = (int64_t)E * NP + a;
        T x[2], v[2];
        node_motion(M.xn[2 * na], M.xn[2 * na + 1], M.wbl[na], cs, sn, mo, x, v);
        sx[e][a][0] = x[0]; sx[e][a][1] = x[1];
        sv[e][a][0] = v[0]; sv[e][a][1] = v[1];
    }
    __syncthreads();
    for (int q = tid; q < NQ; q += blockDim.x) {
        double gx[NP][2];
        grad_X<NP>(M.jit + 4 * K, R->dphq[q], gx);
        T G[2][2], vG[2], cof[2][2], Gi[2][2];
        point_geom<NP, T>(sx[0], sv[0], R->phq[q], gx, G, vG);
        cof_inv(G, cof, Gi);
        sw[q][0] = cof[0][0] * vG[0] + cof[1][0] * vG[1];
        sw[q][1] = cof[0][1] * vG[0] + cof[1][1] * vG[1];
    }
    if (tid < 3 * NF) {
        int f = tid / NF, j = tid % NF;
        bool KL = !(nb[f] >= 0 && nb[f] < K);
        int Ls = KL ? 0 : 1 + f, L = KL ? K : nb[f], fL = KL ? f : tw[f];
        const double* N = M.enrm + 2 * (3 * L + fL);
        double gx[NP][2];
        grad_X<NP>(M.jit + 4 * L, R->dphf[fL][j], gx);
        T G[2][2], vG[2], cof[2][2], Gi[2][2];
        point_geom<NP, T>(sx[Ls], sv[Ls], R->phf[fL][j], gx, G, vG);
        cof_inv(G, cof, Gi);
        T cn0 = cof[0][0] * N[0] + cof[0][1] * N[1];
        T cn1 = cof[1][0] * N[0] + cof[1][1] * N[1];
        sfl[f][j] = (KL ? 1.0 : -1.0) * (vG[0] * cn0 + vG[1] * cn1);
    }
    __syncthreads();
    if (tid < NP) {
        int a = tid;
        const double* jt = M.jit + 4 * K;
        T acc = AD<T>::c(0.0);
        for (int q = 0; q < NQ; ++q) {
            double g0 = jt[0] * R->dphq[q][a][0] + jt[1] * R->dphq[q][a][1];
            double g1 = jt[2] * R->dphq[q][a][0] + jt[3] * R->dphq[q][a][1];
            acc += R->wq[q] * (g0 * sw[q][0] + g1 * sw[q][1]);
        }
        acc = (-2.0 * M.area[K]) * acc;
        for (int f = 0; f < 3; ++f) {
            bool KL = !(nb[f] >= 0 && nb[f] < K);
            T s = AD<T>::c(0.0);
            for (int j = 0; j < NF; ++j) s += (R->wf[j] * (KL ? R->phf[f][j][a] : R->phr[f][j][a])) * sfl[f][j];
            acc += M.elen[3 * K + f] * s;
        }
        int64_t idx = (int64_t)K * NP + a;
        if constexpr (sizeof(T) == sizeof(double)) {
            out[idx] = AD<T>::val(acc);
        } else {
            const double* dd = reinterpret_cast<const double*>(&acc);
            out[idx] = dd[0];
            out[nn + idx] = dd[1];
            out[2 * nn + idx] = dd[2];
            out[3 * nn + idx] = dd[3];
        }
    }
}

// gbar(0): L2 projection of det G at t = 0 (value and mu-derivatives)
template <int P, class T>
__global__ void __launch_bounds__(64) k_gbar0(DevMesh M, const Ref<P>* __restrict__ R, Motion<T> mo,
                                              double* __restrict__ out, int64_t nn)
{
    constexpr int NP = Sz<P>::NP, NQ = Sz<P>::NQ;
    const int K = blockIdx.x, tid = threadIdx.x;
    __shared__ T sx[NP][2], sv[NP][2];
    __shared__ T sdet[NQ];
    T cs, sn;
    dsincos(mo.th, &sn, &cs);
    if (tid < NP) {
        int64_t na = (int64_t)K * NP + tid;
        T x[2], v[2];
        node_motion(M.xn[2 * na], M.xn[2 * na + 1], M.wbl[na], cs, sn, mo, x, v);
        sx[tid][0] = x[0]; sx[tid][1] = x[1];
        sv[tid][0] = v[0]; sv[tid][1] = v[1];
    }
    __syncthreads();
    for (int q = tid; q < NQ; q += blockDim.x) {
        double gx[NP][2];
        grad_X<NP>(M.jit + 4 * K, R->dphq[q], gx);
        T G[2][2], vG[2];
        point_geom<NP, T>(sx, sv, R->phq[q], gx, G, vG);
        sdet[q] = G[0][0] * G[1][1] - G[0][1] * G[1][0];
    }
    __syncthreads();
    if (tid < NP) {
        T acc = AD<T>::c(0.0);
        for (int b = 0; b < NP; ++b) {
            T pb = AD<T>::c(0.0);
            for (int q = 0; q < NQ; ++q) pb += (R->wq[q] * R->phq[q][b]) * sdet[q];
            acc += R->mhi[tid][b] * pb;
        }
        int64_t idx = (int64_t)K * NP + tid;
        if constexpr (sizeof(T) == sizeof(double)) {
            out[idx] = AD<T>::val(acc);
        } else {
            const double* dd = reinterpret_cast<const double*>(&acc);
            out[idx] = dd[0];
            out[nn + idx] = dd[1];
            out[2 * nn + idx] = dd[2];
            out[3 * nn + idx] = dd[3];
        }
    }
}

// kg = dt M^{-1} r_g (per element: mhi / (2|K|)), for value + 3 derivative fields
template <int P>
__global__ void k_gcl_kstage(DevMesh M, const Ref<P>* __restrict__ R, const double* __restrict__ rg, double dt,
                             double* __restrict__ kg, int nfield, int64_t nn)
{
    constexpr int NP = Sz<P>::NP;
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nn * nfield) return;
    int64_t fld = t / nn, idx = t % nn;
    int K = (int)(idx / NP), a = (int)(idx % NP);
    const double* r = rg + fld * nn + (int64_t)K * NP;
    double s = 0.0;
    for (int b = 0; b < NP; ++b) s += R->mhi[a][b] * r[b];
    kg[t] = dt * s / (2.0 * M.area[K]);
}

// ------------------------------------------------------------------ QoI
// Force on the body: momentum part of the wall numerical flux integrated over
// the wall (Sec. 4 eq. qoi, solver-consistent reading); P = f . v_G, F_x = f . e1.
// One thread per (wall element, dual seed): seed < B differentiates w.r.t.
// U_X[K][seed]; outputs per wall element: f [2] and df/du [2][B].
template <int P>
__global__ void k_qoi_du(DevMesh M, const Ref<P>* __restrict__ R, Phys ph, Motion<double> mo,
                         const int32_t* __restrict__ wall_elems, int nwall, const double* __restrict__ u,
                         const double* __restrict__ gb, double* __restrict__ fval, double* __restrict__ dfdu)
{
    constexpr int NP = Sz<P>::NP, NF = Sz<P>::NF, B = Sz<P>::B;
    using D1 = Dual<1>;
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nwall * B) return;
    int w = t / B, sd = t % B;
    int K = wall_elems[w];
    double cs = cos(mo.th), sn = sin(mo.th);
    D1 uu[NP][4];
    double g[NP], x[NP][2], v[NP][2];
    for (int a = 0; a < NP; ++a) {
        int64_t na = (int64_t)K * NP + a;
        for (int m = 0; m < 4; ++m) uu[a][m] = AD<D1>::c(u[na * 4 + m]);
        g[a] = gb[na];
        node_motion(M.xn[2 * na], M.xn[2 * na + 1], M.wbl[na], cs, sn, mo, x[a], v[a]);
    }
    uu[sd >> 2][sd & 3].d[0] = 1.0;
    D1 gD[NP], xD[NP][2], vD[NP][2];
    for (int a = 0; a < NP; ++a) {
        gD[a] = AD<D1>::c(g[a]);
        for (int d = 0; d < 2; ++d) { xD[a][d] = AD<D1>::c(x[a][d]); vD[a][d] = AD<D1>::c(v[a][d]); }
    }
    D1 fP = AD<D1>::c(0.0), fX = AD<D1>::c(0.0);
    for (int f = 0; f < 3; ++f) {
        if (M.enb[3 * K + f] != -1 || M.wall_is_far) continue;
        const double* N = M.enrm + 2 * (3 * K + f);
        double len = M.elen[3 * K + f], hK = 2.0 * M.area[K] / len;
        for (int j = 0; j < NF; ++j) {
            double gx[NP][2];
            grad_X<NP>(M.jit + 4 * K, R->dphf[f][j], gx);
            D1 U[4], gU[4][2], G[2][2], vG[2], Fh[4];
            point_state<NP, D1>(uu, gD, R->phf[f][j], gx, U, gU);
            point_geom<NP, D1>(xD, vD, R->phf[f][j], gx, G, vG);
            bnd_flux(ph, true, hK, U, gU, G, vG, N, Fh);
            double wj = len * R->wf[j];
            fP += wj * (Fh[1] * vG[0] + Fh[2] * vG[1]);
            fX += wj * Fh[1];
        }
    }
    dfdu[((int64_t)w * 2 + 0) * B + sd] = fP.d[0];
    dfdu[((int64_t)w * 2 + 1) * B + sd] = fX.d[0];
    if (sd == 0) {
        fval[2 * w] = fP.v;
        fval[2 * w + 1] = fX.v;
    }
}

// mu-derivative of the QoIs: one thread per wall element, Dual<3> through the
// mesh motion and gbar; out [nwall][2][4] = (value, d/dmu_0..2)
template <int P>
__global__ void k_qoi_dmu(DevMesh M, const Ref<P>* __restrict__ R, Phys ph, Motion<Dual<3>> mo,
                          const int32_t* __restrict__ wall_elems, int nwall, const double* __restrict__ u,
                          const double* __restrict__ gb, const double* __restrict__ dgb, double* __restrict__ out,
                          int64_t nn)
{
    constexpr int NP = Sz<P>::NP, NF = Sz<P>::NF;
    using D3 = Dual<3>;
    int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= nwall) return;
    int K = wall_elems[w];
    D3 cs, sn;
    dsincos(mo.th, &sn, &cs);
    D3 uu[NP][4], g[NP], x[NP][2], v[NP][2];
    for (int a = 0; a < NP; ++a) {
        int64_t na = (int64_t)K * NP + a;
        for (int m = 0; m < 4; ++m) uu[a][m] = AD<D3>::c(u[na * 4 + m]);
        g[a] = load_g<D3>(gb, dgb, na, nn);
        node_motion(M.xn[2 * na], M.xn[2 * na + 1], M.wbl[na], cs, sn, mo, x[a], v[a]);
    }
    D3 fP = AD<D3>::c(0.0), fX = AD<D3>::c(0.0);
    for (int f = 0; f < 3; ++f) {
        if (M.enb[3 * K + f] != -1 || M.wall_is_far) continue;
        const double* N = M.enrm + 2 * (3 * K + f);
        double len = M.elen[3 * K + f], hK = 2.0 * M.area[K] / len;
        for (int j = 0; j < NF; ++j) {
            double gx[NP][2];
            grad_X<NP>(M.jit + 4 * K, R->dphf[f][j], gx);
            D3 U[4], gU[4][2], G[2][2], vG[2], Fh[4];
            point_state<NP, D3>(uu, g, R->phf[f][j], gx, U, gU);
            point_geom<NP, D3>(x, v, R->phf[f][j], gx, G, vG);
            bnd_flux(ph, true, hK, U, gU, G, vG, N, Fh);
            double wj = len * R->wf[j];
            fP += wj * (Fh[1] * vG[0] + Fh[2] * vG[1]);
            fX += wj * Fh[1];
        }
    }
    double* o = out + (int64_t)w * 8;
    o[0] = fP.v; o[1] = fP.d[0]; o[2] = fP.d[1]; o[3] = fP.d[2];
    o[4] = fX.v; o[5] = fX.d[0]; o[6] = fX.d[1]; o[7] = fX.d[2];
}

}  // namespace pa
