// Host orchestration and C ABI of the periodic-adjoint library (gfx950).
//
// Implements, on one MI355X, the fully discrete time-periodic adjoint method
// of arXiv:1512.00616:
//   primal period (Sec. 2.2 eq. dirk2): per DIRK stage a Newton solve with
//     the exact Jacobian and block-Jacobi GMRES;
//   tangent sweep (eq. dirk-sens-mvp) = matvec of Newton-Krylov shooting
//     (Alg. 2, Jacobian Phi - I of eq. jac-prim);
//   backward adjoint sweep (eqs. uns-disc-adj-dirk2 and
//     uns-disc-adj-dirk-sens-mvp) with transposed stage solves;
//   periodic adjoint GMRES (Alg. 3) and the gradient (eq.
//     funcl-grad-nosens-dirk, Alg. 4).
// Every stage state, stage slope, Jacobian and block-Jacobi inverse of the
// period is checkpointed in HBM during the primal sweep, so the tangent and
// adjoint sweeps only stream stored operators.
#include "../../include/pa.h"
#include "pa_kernels.hpp"
#include "pa_linalg.hpp"
#include "pa_learn.hpp"

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <string>
#include <vector>
#include <thread>
#include <atomic>
#include <mutex>

using namespace pa;

namespace {

struct PaError {
    pa_status code;
    std::string msg;
};

[[noreturn]] void raise(pa_status c, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    throw PaError{ c, buf };
}

#define HIPCHK(expr)                                                                                 \
    do {                                                                                             \
        hipError_t e_ = (expr);                                                                      \
        if (e_ != hipSuccess) raise(PA_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));      \
    } while (0)

#define LAUNCHCHK()                                                                                  \
    do {                                                                                             \
        hipError_t e_ = hipGetLastError();                                                           \
        if (e_ != hipSuccess) raise(PA_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e_));   \
    } while (0)

double now_ms()
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ------------------------------------------------------------------ reference element (host)
// Gauss-Legendre rule on [0, 1] by Newton's method on P_n
void gauss_legendre01(int n, std::vector<double>& x, std::vector<double>& w)
{
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int k = 0; k < n; ++k) {
        double z = -std::cos(M_PI * (k + 0.75) / (n + 0.5));   // ascending
        double dpn = 1.0;
        for (int it = 0; it < 100; ++it) {
            double pm = 1.0, pc = z;   // P_0, P_1
            for (int l = 2; l <= n; ++l) {
                double pn = ((2 * l - 1) * z * pc - (l - 1) * pm) / l;
                pm = pc;
                pc = pn;
            }
            dpn = n * (pm - z * pc) / (1.0 - z * z);
            double step = pc / dpn;
            z -= step;
            if (std::fabs(step) < 1e-17) break;
        }
        double pm = 1.0, pc = z;
        for (int l = 2; l <= n; ++l) {
            double pn = ((2 * l - 1) * z * pc - (l - 1) * pm) / l;
            pm = pc;
            pc = pn;
        }
        dpn = n * (pm - z * pc) / (1.0 - z * z);
        x[k] = 0.5 * (z + 1.0);
        w[k] = 1.0 / ((1.0 - z * z) * dpn * dpn);
    }
}

// Lagrange basis on the equispaced nodal set via a monomial Vandermonde
// matrix inverted by Gauss-Jordan elimination
struct Basis {
    int p, np;
    std::vector<int> ex, ey;
    std::vector<double> coef;   // coef[k*np + a]: phi_a = sum_k coef * monomial_k
    explicit Basis(int p_) : p(p_), np((p_ + 1) * (p_ + 2) / 2)
    {
        for (int i = 0; i <= p; ++i)
            for (int j = 0; i + j <= p; ++j) { ex.push_back(i); ey.push_back(j); }
        std::vector<double> nodes;
        for (int t = 0; t <= p; ++t)
            for (int s = 0; s + t <= p; ++s) { nodes.push_back((double)s / p); nodes.push_back((double)t / p); }
        // augmented [V | I], V[b][k] = monomial_k(node_b)
        int n = np;
        std::vector<double> a(n * 2 * n, 0.0);
        for (int b = 0; b < n; ++b) {
            for (int k = 0; k < n; ++k) a[b * 2 * n + k] = std::pow(nodes[2 * b], ex[k]) * std::pow(nodes[2 * b + 1], ey[k]);
            a[b * 2 * n + n + b] = 1.0;
        }
        for (int c = 0; c < n; ++c) {
            int piv = c;
            for (int r = c + 1; r < n; ++r)
                if (std::fabs(a[r * 2 * n + c]) > std::fabs(a[piv * 2 * n + c])) piv = r;
            if (piv != c)
                for (int k = 0; k < 2 * n; ++k) std::swap(a[c * 2 * n + k], a[piv * 2 * n + k]);
            double d = a[c * 2 * n + c];
            for (int k = 0; k < 2 * n; ++k) a[c * 2 * n + k] /= d;
            for (int r = 0; r < n; ++r) {
                if (r == c) continue;
                double f = a[r * 2 * n + c];
                if (f != 0.0)
                    for (int k = 0; k < 2 * n; ++k) a[r * 2 * n + k] -= f * a[c * 2 * n + k];
            }
        }
        // V^{-1} = right half; coef[k][a] = Vinv[k][a]
        coef.assign(n * n, 0.0);
        for (int k = 0; k < n; ++k)
            for (int b = 0; b < n; ++b) coef[k * n + b] = a[k * 2 * n + n + b];
    }
    void eval(double x, double y, double* phi, double (*dphi)[2]) const
    {
        for (int a = 0; a < np; ++a) { phi[a] = 0.0; dphi[a][0] = dphi[a][1] = 0.0; }
        for (int k = 0; k < np; ++k) {
            double m = std::pow(x, ex[k]) * std::pow(y, ey[k]);
            double mx = ex[k] ? ex[k] * std::pow(x, ex[k] - 1) * std::pow(y, ey[k]) : 0.0;
            double my = ey[k] ? ey[k] * std::pow(x, ex[k]) * std::pow(y, ey[k] - 1) : 0.0;
            for (int a = 0; a < np; ++a) {
                double c = coef[k * np + a];
                phi[a] += c * m;
                dphi[a][0] += c * mx;
                dphi[a][1] += c * my;
            }
        }
    }
};

template <int P>
void build_ref(Ref<P>& R)
{
    constexpr int NP = Sz<P>::NP, NF = Sz<P>::NF;
    Basis bs(P);
    std::vector<double> gx, gw;
    gauss_legendre01(P + 2, gx, gw);
    int q = 0;
    for (int l = 0; l < P + 2; ++l)
        for (int k = 0; k < P + 2; ++k) {
            double xi = gx[k] * (1.0 - gx[l]), eta = gx[l];
            bs.eval(xi, eta, R.phq[q], R.dphq[q]);
            R.wq[q] = gw[k] * gw[l] * (1.0 - gx[l]);
            ++q;
        }
    const double rv[3][2] = { { 0, 0 }, { 1, 0 }, { 0, 1 } };
    for (int f = 0; f < 3; ++f)
        for (int j = 0; j < NF; ++j) {
            const double *a = rv[f], *b = rv[(f + 1) % 3];
            double s = gx[j], sr = 1.0 - gx[j];
            bs.eval(a[0] + s * (b[0] - a[0]), a[1] + s * (b[1] - a[1]), R.phf[f][j], R.dphf[f][j]);
            bs.eval(a[0] + sr * (b[0] - a[0]), a[1] + sr * (b[1] - a[1]), R.phr[f][j], R.dphr[f][j]);
        }
    for (int j = 0; j < NF; ++j) R.wf[j] = gw[j];
    for (int a = 0; a < NP; ++a)
        for (int b = 0; b < NP; ++b) {
            double s = 0.0;
            for (int qq = 0; qq < Sz<P>::NQ; ++qq) s += R.wq[qq] * R.phq[qq][a] * R.phq[qq][b];
            R.mh[a][b] = s;
        }
    // inverse of the mass matrix (Gauss-Jordan)
    int n = NP;
    std::vector<double> a(n * 2 * n, 0.0);
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j) a[i * 2 * n + j] = R.mh[i][j];
        a[i * 2 * n + n + i] = 1.0;
    }
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(a[r * 2 * n + c]) > std::fabs(a[piv * 2 * n + c])) piv = r;
        if (piv != c)
            for (int k = 0; k < 2 * n; ++k) std::swap(a[c * 2 * n + k], a[piv * 2 * n + k]);
        double d = a[c * 2 * n + c];
        for (int k = 0; k < 2 * n; ++k) a[c * 2 * n + k] /= d;
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            double f = a[r * 2 * n + c];
            for (int k = 0; k < 2 * n; ++k) a[r * 2 * n + k] -= f * a[c * 2 * n + k];
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) R.mhi[i][j] = a[i * 2 * n + n + j];
}

// Alexander's three-stage, L-stable, stiffly accurate DIRK of order 3
// (reading of the third-order DIRK of Sec. 4.1; the paper gives no tableau)
struct Dirk3 {
    double A[3][3], b[3], c[3];
    Dirk3()
    {
        // alpha: root in (1/6, 1/2) of x^3 - 3x^2 + 3x/2 - 1/6, by bisection
        double lo = 1.0 / 6.0, hi = 0.5;
        for (int it = 0; it < 200; ++it) {
            double mid = 0.5 * (lo + hi);
            double f = ((mid - 3.0) * mid + 1.5) * mid - 1.0 / 6.0;
            double flo = ((lo - 3.0) * lo + 1.5) * lo - 1.0 / 6.0;
            if ((f < 0) == (flo < 0)) lo = mid; else hi = mid;
        }
        double al = 0.5 * (lo + hi), t2 = 0.5 * (1.0 + al);
        double b1 = -(6 * al * al - 16 * al + 1) / 4.0, b2 = (6 * al * al - 20 * al + 5) / 4.0;
        std::memset(A, 0, sizeof A);
        A[0][0] = al;
        A[1][0] = t2 - al; A[1][1] = al;
        A[2][0] = b1; A[2][1] = b2; A[2][2] = al;
        b[0] = b1; b[1] = b2; b[2] = al;
        c[0] = al; c[1] = t2; c[2] = 1.0;
    }
};

inline int grid1(int64_t n, int bs = 256) { return (int)((n + bs - 1) / bs); }

// Multilayer perceptron on the device (FP32): widths dims[0] -> ... -> dims[L],
// tanh on hidden layers, linear output, parameters flat [W_1 b_1 W_2 b_2 ...]
// with W_l [dims[l]][dims[l-1]] row-major; batches column-major [feature][sample].
// Device memory of a context: the caller's callbacks (pa_config dev_alloc /
// dev_free) when both are given, else hipMalloc / hipFree.
struct DevAlloc {
    void* (*fa)(uint64_t, void*) = nullptr;
    void (*ff)(void*, void*) = nullptr;
    void* user = nullptr;
    void* get(size_t bytes) const
    {
        if (bytes == 0) bytes = 1;
        if (fa && ff) {
            void* q = fa((uint64_t)bytes, user);
            if (!q) raise(PA_ENOMEM, "device allocation callback returned NULL for %.3f GB", bytes / 1e9);
            return q;
        }
        void* q = nullptr;
        const hipError_t e = hipMalloc(&q, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            raise(PA_ENOMEM, "hipMalloc of %.3f GB failed: %s", bytes / 1e9, hipGetErrorString(e));
        }
        return q;
    }
    void put(void* q) const
    {
        if (!q) return;
        if (fa && ff) ff(q, user);
        else (void)hipFree(q);
    }
};

// Shape of the perceptron in -> w -> w -> w -> out: parameter offsets in the
// flat layout [W1 b1 W2 b2 W3 b3 W4 b4] (W_l row-major [out_l][in_l]).
struct MlpShape {
    int dims[5] = { 0, 0, 0, 0, 0 };
    int64_t woff[4] = { 0, 0, 0, 0 }, boff[4] = { 0, 0, 0, 0 };
    int64_t nparam = 0;
    int maxw = 0;
    MlpShape() = default;
    MlpShape(int in, int width, int out)
    {
        const int d[5] = { in, width, width, width, out };
        for (int l = 0; l < 5; ++l) dims[l] = d[l];
        for (int l = 0; l < 4; ++l) {
            woff[l] = nparam;
            nparam += (int64_t)dims[l + 1] * dims[l];
            boff[l] = nparam;
            nparam += dims[l + 1];
            maxw = std::max(maxw, std::max(dims[l], dims[l + 1]));
        }
    }
};

// One pass of the perceptron on raw device buffers (no allocation): forward
// into the activations H[0..3] ([dims[l+1]][S]), the mean squared error
// against T with dY in dA, and the gradients into g (dA, dB [maxw][S] are
// work buffers).
inline void mlp_gemm(int M, int N, int K, const float* A, int tA, const float* B, int tB, float* C, hipStream_t st)
{
    dim3 grid((N + GT - 1) / GT, (M + GT - 1) / GT);
    k_gemm_mfma_f32<<<grid, 64, 0, st>>>(M, N, K, A, tA, B, tB, C);
    LAUNCHCHK();
}
inline void mlp_forward(const MlpShape& sh, const float* p, const float* X, float* const H[4], int S, hipStream_t st)
{
    const float* in = X;
    for (int l = 0; l < 4; ++l) {
        mlp_gemm(sh.dims[l + 1], S, sh.dims[l], p + sh.woff[l], 0, in, 0, H[l], st);
        k_bias_act<<<grid1((int64_t)sh.dims[l + 1] * S), 256, 0, st>>>(H[l], p + sh.boff[l], sh.dims[l + 1], S, l < 3);
        LAUNCHCHK();
        in = H[l];
    }
}
inline void mlp_mse(const MlpShape& sh, const float* const H[4], const float* T, float* dA, int S, float* loss,
                    hipStream_t st)
{
    k_mse<<<1, 256, 0, st>>>(H[3], T, dA, (int64_t)sh.dims[4] * S, loss);
    LAUNCHCHK();
}
inline void mlp_backward(const MlpShape& sh, const float* p, const float* X, const float* const H[4], float* dA,
                         float* dB, float* g, int S, hipStream_t st)
{
    float* cur = dA;
    for (int l = 3; l >= 0; --l) {
        const float* in = l == 0 ? X : H[l - 1];
        mlp_gemm(sh.dims[l + 1], sh.dims[l], S, cur, 0, in, 1, g + sh.woff[l], st);
        k_row_sum<<<grid1(sh.dims[l + 1]), 256, 0, st>>>(cur, g + sh.boff[l], sh.dims[l + 1], S);
        LAUNCHCHK();
        if (l > 0) {
            float* nxt = cur == dA ? dB : dA;
            mlp_gemm(sh.dims[l], S, sh.dims[l + 1], p + sh.woff[l], 1, cur, 0, nxt, st);
            k_tanh_back<<<grid1((int64_t)sh.dims[l] * S), 256, 0, st>>>(nxt, H[l - 1], (int64_t)sh.dims[l] * S);
            LAUNCHCHK();
            cur = nxt;
        }
    }
}

struct Mlp {
    MlpShape sh;
    int64_t nparam = 0;
    int cap = 0;
    float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
    float *X = nullptr, *T = nullptr, *dA = nullptr, *dB = nullptr, *loss = nullptr;
    float* H[4] = { nullptr, nullptr, nullptr, nullptr };
    hipStream_t st = nullptr;
    int step = 0;
    DevAlloc da;
    void fr(float*& q) { da.put(q); q = nullptr; }
    float* al(int64_t n) { return static_cast<float*>(da.get(sizeof(float) * (size_t)std::max<int64_t>(n, 1))); }
    void release()
    {
        fr(p); fr(g); fr(m); fr(v); fr(X); fr(T); fr(dA); fr(dB); fr(loss);
        for (auto& h : H) fr(h);
        cap = 0;
    }
    ~Mlp() { release(); }
    int width() const { return sh.dims[1]; }
    void init(int in, int width, int out, hipStream_t s)
    {
        release();
        sh = MlpShape(in, width, out);
        nparam = sh.nparam;
        st = s;
        step = 0;
        p = al(nparam); g = al(nparam); m = al(nparam); v = al(nparam);
        HIPCHK(hipMemsetAsync(m, 0, sizeof(float) * nparam, st));
        HIPCHK(hipMemsetAsync(v, 0, sizeof(float) * nparam, st));
        loss = al(1);
    }
    void reserve(int batch)
    {
        if (batch <= cap) return;
        for (auto& h : H) fr(h);
        fr(X); fr(T); fr(dA); fr(dB);
        for (int l = 0; l < 4; ++l) H[l] = al((int64_t)sh.dims[l + 1] * batch);
        X = al((int64_t)sh.dims[0] * batch);
        T = al((int64_t)sh.dims[4] * batch);
        dA = al((int64_t)sh.maxw * batch);
        dB = al((int64_t)sh.maxw * batch);
        cap = batch;
    }
    const float* out() const { return H[3]; }
    void forward(int S) { mlp_forward(sh, p, X, H, S, st); }
    // loss and dY = d loss / d output into dA
    void mse(int S) { mlp_mse(sh, H, T, dA, S, loss, st); }
    // gradients into g from dY in dA (after forward and mse)
    void backward(int S) { mlp_backward(sh, p, X, H, dA, dB, g, S, st); }
    void adam(float lr)
    {
        ++step;
        const float b1 = 0.9f, b2 = 0.999f;
        const float c1 = 1.0f - std::pow(b1, (float)step), c2 = 1.0f - std::pow(b2, (float)step);
        k_adam<<<grid1(nparam), 256, 0, st>>>(p, g, m, v, nparam, lr, b1, b2, 1e-8f, c1, c2);
        LAUNCHCHK();
    }
};

// eigenvalues of an upper Hessenberg matrix (n x n, row-major) by the
// shifted QR algorithm in complex arithmetic (Wilkinson shift, deflation of
// negligible subdiagonals); the matrix is overwritten
inline void hess_eig(std::vector<std::complex<double>>& H, int n, std::vector<std::complex<double>>& ev)
{
    using cd = std::complex<double>;
    ev.assign(n, cd(0, 0));
    auto at = [&](int i, int j) -> cd& { return H[(size_t)i * n + j]; };
    int hi = n - 1, iter = 0;
    while (hi >= 0) {
        if (hi == 0) { ev[0] = at(0, 0); break; }
        // find the active block [lo, hi]
        int lo = hi;
        while (lo > 0) {
            const double sub = std::abs(at(lo, lo - 1));
            const double dia = std::abs(at(lo, lo)) + std::abs(at(lo - 1, lo - 1));
            if (sub <= 1e-15 * (dia > 0 ? dia : 1.0)) { at(lo, lo - 1) = 0; break; }
            --lo;
        }
        if (lo == hi) { ev[hi] = at(hi, hi); --hi; iter = 0; continue; }
        if (++iter > 100 * n) raise(PA_ENOCONV, "Hessenberg QR did not converge");
        // Wilkinson shift from the trailing 2 x 2 block (exceptional shift now and then)
        const cd a = at(hi - 1, hi - 1), b = at(hi - 1, hi), c = at(hi, hi - 1), d = at(hi, hi);
        const cd tr = a + d, det = a * d - b * c;
        const cd disc = std::sqrt(tr * tr - 4.0 * det);
        const cd l1 = 0.5 * (tr + disc), l2 = 0.5 * (tr - disc);
        cd mu = std::abs(l1 - d) < std::abs(l2 - d) ? l1 : l2;
        if (iter % 11 == 0) mu += cd(std::abs(at(hi, hi - 1)), 0.0);
        // QR step on the block by Givens rotations: H - mu I = Q R, H <- R Q + mu I
        std::vector<cd> cs(hi - lo), sn(hi - lo);
        for (int k = lo; k <= hi; ++k) at(k, k) -= mu;
        for (int k = lo; k < hi; ++k) {
            const cd x = at(k, k), y = at(k + 1, k);
            const double r = std::sqrt(std::norm(x) + std::norm(y));
            const cd cc = r > 0 ? x / r : cd(1, 0), ss = r > 0 ? y / r : cd(0, 0);
            cs[k - lo] = cc;
            sn[k - lo] = ss;
            for (int j = k; j < n; ++j) {   // rows k, k+1 <- G^H rows
                const cd u = at(k, j), v = at(k + 1, j);
                at(k, j) = std::conj(cc) * u + std::conj(ss) * v;
                at(k + 1, j) = -ss * u + cc * v;
            }
        }
        for (int k = lo; k < hi; ++k) {     // columns k, k+1 <- columns G
            const cd cc = cs[k - lo], ss = sn[k - lo];
            for (int i = 0; i <= std::min(k + 1, hi); ++i) {
                const cd u = at(i, k), v = at(i, k + 1);
                at(i, k) = u * cc + v * ss;
                at(i, k + 1) = -u * std::conj(ss) + v * std::conj(cc);
            }
        }
        for (int k = lo; k <= hi; ++k) at(k, k) += mu;
    }
}

// splitmix64: seeded initial weights
inline uint64_t splitmix64(uint64_t& x)
{
    uint64_t z = (x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// eigenpairs of a symmetric n x n matrix (row-major, destroyed) by cyclic
// Jacobi rotations; eigenvalues descending in w, eigenvectors as columns of V
inline void sym_eig(std::vector<double>& A, int n, std::vector<double>& w, std::vector<double>& V)
{
    V.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                const double a = A[(size_t)i * n + j] * A[(size_t)i * n + j];
                tot += a;
                if (i != j) off += a;
            }
        if (off <= 1e-30 * tot) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = A[(size_t)p * n + q];
                if (std::fabs(apq) < 1e-300) continue;
                const double app = A[(size_t)p * n + p], aqq = A[(size_t)q * n + q];
                const double th = (aqq - app) / (2.0 * apq);
                const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {   // columns p, q
                    const double akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
                    A[(size_t)k * n + p] = c * akp - s * akq;
                    A[(size_t)k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {   // rows p, q
                    const double apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
                    A[(size_t)p * n + k] = c * apk - s * aqk;
                    A[(size_t)q * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    const double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
                    V[(size_t)k * n + p] = c * vkp - s * vkq;
                    V[(size_t)k * n + q] = s * vkp + c * vkq;
                }
            }
    }
    std::vector<int> idx(n);
    for (int i = 0; i < n; ++i) idx[i] = i;
    std::sort(idx.begin(), idx.end(), [&](int a, int b) { return A[(size_t)a * n + a] > A[(size_t)b * n + b]; });
    std::vector<double> V2((size_t)n * n);
    w.assign(n, 0.0);
    for (int j = 0; j < n; ++j) {
        w[j] = A[(size_t)idx[j] * n + idx[j]];
        for (int k = 0; k < n; ++k) V2[(size_t)k * n + j] = V[(size_t)k * n + idx[j]];
    }
    V.swap(V2);
}

}  // namespace

// ------------------------------------------------------------------ context
struct pa_ctx {
    pa_config cfg;
    std::string err;
    DevAlloc da;
    virtual ~pa_ctx() {}
    virtual int64_t num_dofs() const = 0;
    virtual int32_t num_elems() const = 0;
    virtual int32_t block_size() const = 0;
    virtual int64_t device_bytes() const = 0;
    virtual int64_t kernel_vectors(int k) = 0;
    virtual void get_mesh(int32_t*, int32_t*, int8_t*, double*) const = 0;
    virtual void set_params(const double mu[3]) = 0;
    virtual void set_state(const double* u0, int64_t n) = 0;
    virtual void set_freestream(const double* pert) = 0;
    virtual void get_state(int which, double* out, int64_t n) = 0;
    virtual void primal_period(double qoi[2], double* res) = 0;
    virtual void last_qois(double q[2]) const = 0;
    void optimize(const pa_opt_opts& o, double mu[3], pa_opt_report* rep);
    virtual void shoot(double tol, double eta, int maxit, pa_shoot_report* rep) = 0;
    virtual void fixed_point(int periods, double* res) = 0;
    virtual void shoot_descent(double tol, int memory, int maxit, pa_shoot_report* rep) = 0;
    virtual double periodicity_gradient(double* grad) = 0;
    virtual int floquet(int k, uint64_t seed, double* re, double* im, double* hsub) = 0;
    virtual void adjoint_gradient(double rtol, double qoi[2], double dJ[6], pa_adjoint_report* rep) = 0;
    virtual void tangent_gradient(double rtol, double dJ[6], int32_t its[3]) = 0;
    virtual void ws_train(const double* params, const double* states, int S, const pa_ws_opts& o, double* loss) = 0;
    virtual void ws_predict(const double m[3]) = 0;
    virtual void ws_shoot(double tol, double eta, int maxit, pa_shoot_report* rep, int32_t* fell_back) = 0;
    virtual void ws_save(const char* path) = 0;
    virtual int ws_pod(int kmax, double* mean, double* modes, double* eig) = 0;
    virtual void node_coords(double* xy) const = 0;
    virtual void ws_load(const char* path) = 0;
    virtual void tangent_sweep_h(const double* v, double* out) = 0;
    virtual void adjoint_sweep_h(const double* lam, int fq, double* lam0, double* grad) = 0;
    virtual void dbg_gbar(int n, int i, double* out, bool deriv) = 0;
    virtual void dbg_residual(int n, int i, const double* u, double* r, bool dmu) = 0;
    virtual void dbg_jacobian(int n, int i, const double* u, double* blk) = 0;
    virtual void dbg_qoi(int n, int i, const double* u, double f[2], double* dfdu, double* dfdmu) = 0;
    virtual void dbg_bsr_apply(const double* blk, double alpha, double beta, int tr, const double* x, double* y) = 0;
    virtual void dbg_blockinv(const double* blk, double adt, double* out) = 0;
    virtual int dbg_stage_solve(const double* blk, double adt, int tr, const double* rhs, double* x) = 0;
    virtual void dbg_traj(int which, int n, int i, double* out) = 0;
    virtual void set_timing(bool on) = 0;
    virtual void kernel_time(int k, double* ms, int64_t* cnt) = 0;
    virtual int64_t kernel_skipped(int k) = 0;
    virtual double bench_spmv(int reps, int tr) = 0;
    virtual double bench_spmv_m(int reps, int tr, int R) = 0;
    virtual double bench_spmv_lo(int reps, int tr) = 0;
    virtual void tuning(int32_t* q, double us[3]) = 0;
    virtual double bench_copy(int reps, int64_t* bytes) = 0;
};

namespace {

template <int P>
struct Solver final : pa_ctx {
    static constexpr int NP = Sz<P>::NP, NQ = Sz<P>::NQ, NF = Sz<P>::NF, B = Sz<P>::B, BB = B * B;
    // stored operators of one stage: Ahat = A P^{-1} (off-diagonal blocks),
    // P = diagonal blocks of A = M - aii J, and P^{-1}
    struct StageOps {
        const double *Ah, *Pd, *Pinv;
        double aii;        // dt a_ii of the stage
        const void* Al;    // low-precision copy of Ah (mixed-precision modes)
    };
    struct GmHost { double res; int done; int its; };   // mirrors GmState::res, done, its

    int Ne = 0, Nt = 0, nst = 0, nwall = 0;
    int64_t Nu = 0, nn = 0, Jsz = 0, Isz = 0;
    double dt = 0;
    Dirk3 rk;
    Phys ph{};
    double mu[3] = { 0, 0, 0 };
    bool have_params = false, have_traj = false;
    int restart = 30, max_kry = 100;
    int pmode = PA_PREC_FP64;                                      // stage-solve precision
    void* tAl = nullptr;                                           // low-precision Ahat copies [nst][Ne][3][B][B]
    float *V32 = nullptr, *w32 = nullptr, *r32 = nullptr;          // FP32 inner Krylov basis and vectors
    int verbose = 0;   // PA_VERBOSE=1: solver progress on stderr, 2: also per-stage Newton history
    int64_t bytes = 0;

    // host mesh
    std::vector<int32_t> ev, enb, wall;
    std::vector<int8_t> etw;
    std::vector<double> vxy, area, jit, xn, wbl, elen, enrm;
    Ref<P> href{};

    hipStream_t st = nullptr;
    bool own_stream = false;
    DevMesh dm{};
    const int4 *nb4f = nullptr, *nb4t = nullptr;   // face tables of the applies
    Ref<P>* dref = nullptr;
    double* dmh = nullptr;
    int32_t* dwall = nullptr;
    int* dstatus = nullptr;
    std::vector<void*> allocs;

    double *gb = nullptr, *dgb = nullptr;                          // [(nst+1)][nn], [(nst+1)][3][nn]
    double *tu = nullptr, *tk = nullptr, *tui = nullptr;           // trajectory
    double *tAh = nullptr, *tPd = nullptr, *tAi = nullptr;         // stage operators: Ahat, P, P^{-1}
    double *Jtmp = nullptr;                                        // dr/du of the stage being assembled
    double *qh = nullptr;                                          // [nst][nwall][2]
    double *u0 = nullptr;
    // work vectors
    double *wa = nullptr, *wb = nullptr, *wc = nullptr, *wd = nullptr, *we = nullptr, *wf = nullptr;
    double *sk3 = nullptr;                                         // 3 * Nu
    double *fp3 = nullptr;                                         // 3 * Nu (QoI derivatives)
    double *drm = nullptr;                                         // 3 * Nu (dr/dmu)
    double *V = nullptr, *Vo = nullptr;                            // stage / outer Krylov bases
    double *part = nullptr, *hdev = nullptr;                       // multi-dot partials / results
    double *qtmp = nullptr, *qdu = nullptr, *qdmu = nullptr;
    double *rg4 = nullptr, *kg4 = nullptr;                         // GCL work [3][4][nn]
    int64_t cnt_newton = 0, cnt_gmres = 0;
    int64_t cnt_guess_try = 0, cnt_guess_used = 0;   // stage solves offered an initial guess / that kept it

    // timing
    bool timing = false;
    struct EvPair { hipEvent_t a, b; int k; };
    std::vector<EvPair> evpool;
    size_t evused = 0;
    double ktime[PA_K_COUNT] = { 0 };
    int64_t kcount[PA_K_COUNT] = { 0 };

    template <class T>
    T* dalloc(int64_t n)
    {
        if (n <= 0) n = 1;
        void* p = da.get(sizeof(T) * (size_t)n);
        allocs.push_back(p);
        bytes += sizeof(T) * n;
        return static_cast<T*>(p);
    }

    explicit Solver(const pa_config& c)
    {
        cfg = c;
        da.fa = c.dev_alloc;
        da.ff = c.dev_free;
        da.user = c.user;
        mlp.da = da;
        HIPCHK(hipSetDevice(c.device));
        if (c.stream) st = static_cast<hipStream_t>(c.stream);
        else {
            HIPCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
            own_stream = true;
        }
        Nt = c.Nt;
        nst = 3 * Nt;
        dt = c.T / c.Nt;
        restart = c.gmres_restart;
        pmode = c.precision;
        max_kry = c.max_krylov;
        ph.gam = c.gamma;
        ph.muv = 1.0 / c.re;
        ph.pr = c.pr;
        double pinf = 1.0 / (c.gamma * c.mach * c.mach);
        ph.Uinf[0] = 1.0; ph.Uinf[1] = 1.0; ph.Uinf[2] = 0.0; ph.Uinf[3] = pinf / (c.gamma - 1.0) + 0.5;
        ph.lf_delta = 1e-2;
        ph.wall_eta = 10.0;
        const char* ve = std::getenv("PA_VERBOSE");
        verbose = ve ? std::atoi(ve) : 0;
        build_mesh();
        build_ref(href);
        upload();
    }

    ~Solver() override
    {
        if (st) (void)hipStreamSynchronize(st);
        free_graphs();
        for (auto& e : evpool) { (void)hipEventDestroy(e.a); (void)hipEventDestroy(e.b); }
        for (void* p : allocs) da.put(p);
        if (hstat) (void)hipHostFree(hstat);
        if (hstm) (void)hipHostFree(hstm);
        if (hwgst) (void)hipHostFree(hwgst);
        for (auto& e : gm_ev)
            if (e) (void)hipEventDestroy(e);
        if (st && own_stream) (void)hipStreamDestroy(st);
    }

    // O-grid around the unit circle: radii 1 + (r_far - 1)(q^i - 1)/(q^Nr - 1),
    // q = stretch^(8/Nr); quad (i, j) -> triangles (a, b, c), (a, c, d)
    void build_mesh()
    {
        const int Nr = cfg.Nr, Nth = cfg.Nth;
        Ne = 2 * Nr * Nth;
        nn = (int64_t)Ne * NP;
        Nu = nn * 4;
        Jsz = (int64_t)Ne * 4 * BB;
        Isz = (int64_t)Ne * BB;
        vxy.resize(2 * (Nr + 1) * Nth);
        const double q = std::pow(cfg.stretch, 8.0 / Nr), qN = std::pow(q, Nr);
        for (int i = 0; i <= Nr; ++i) {
            double r = 1.0 + (cfg.r_far - 1.0) * (std::pow(q, i) - 1.0) / (qN - 1.0);
            for (int j = 0; j < Nth; ++j) {
                double th = 2.0 * M_PI * j / Nth;
                vxy[2 * (i * Nth + j)] = r * std::cos(th);
                vxy[2 * (i * Nth + j) + 1] = r * std::sin(th);
            }
        }
        ev.assign(3 * Ne, 0);
        enb.assign(3 * Ne, 0);
        etw.assign(3 * Ne, 0);
        auto wrap = [&](int j) { return ((j % Nth) + Nth) % Nth; };
        auto vid = [&](int i, int j) { return i * Nth + wrap(j); };
        auto eA = [&](int i, int j) { return 2 * (i * Nth + wrap(j)); };
        for (int i = 0; i < Nr; ++i)
            for (int j = 0; j < Nth; ++j) {
                int A = eA(i, j), Bt = A + 1;
                int a = vid(i, j), b = vid(i + 1, j), cc = vid(i + 1, j + 1), d = vid(i, j + 1);
                int* eA3 = &ev[3 * A];
                int* eB3 = &ev[3 * Bt];
                eA3[0] = a; eA3[1] = b; eA3[2] = cc;
                eB3[0] = a; eB3[1] = cc; eB3[2] = d;
                // triangle A: faces a-b, b-c, c-a
                enb[3 * A + 0] = eA(i, j - 1) + 1; etw[3 * A + 0] = 1;
                if (i + 1 < Nr) { enb[3 * A + 1] = eA(i + 1, j) + 1; etw[3 * A + 1] = 2; }
                else { enb[3 * A + 1] = -2; etw[3 * A + 1] = -1; }
                enb[3 * A + 2] = Bt; etw[3 * A + 2] = 0;
                // triangle B: faces a-c, c-d, d-a
                enb[3 * Bt + 0] = A; etw[3 * Bt + 0] = 2;
                enb[3 * Bt + 1] = eA(i, j + 1); etw[3 * Bt + 1] = 0;
                if (i > 0) { enb[3 * Bt + 2] = eA(i - 1, j); etw[3 * Bt + 2] = 1; }
                else { enb[3 * Bt + 2] = -1; etw[3 * Bt + 2] = -1; }
            }
        area.resize(Ne);
        jit.resize(4 * Ne);
        xn.resize(2 * nn);
        wbl.resize(nn);
        elen.resize(3 * Ne);
        enrm.resize(6 * Ne);
        for (int K = 0; K < Ne; ++K) {
            const double* p0 = &vxy[2 * ev[3 * K]];
            const double* p1 = &vxy[2 * ev[3 * K + 1]];
            const double* p2 = &vxy[2 * ev[3 * K + 2]];
            double j00 = p1[0] - p0[0], j01 = p2[0] - p0[0], j10 = p1[1] - p0[1], j11 = p2[1] - p0[1];
            double det = j00 * j11 - j01 * j10;
            area[K] = 0.5 * det;
            // J^{-T} = [[j11, -j10], [-j01, j00]] / det
            jit[4 * K + 0] = j11 / det;
            jit[4 * K + 1] = -j10 / det;
            jit[4 * K + 2] = -j01 / det;
            jit[4 * K + 3] = j00 / det;
            int a = 0;
            for (int t = 0; t <= P; ++t)
                for (int s = 0; s + t <= P; ++s) {
                    double X = p0[0] + (double(s) / P) * (p1[0] - p0[0]) + (double(t) / P) * (p2[0] - p0[0]);
                    double Y = p0[1] + (double(s) / P) * (p1[1] - p0[1]) + (double(t) / P) * (p2[1] - p0[1]);
                    int64_t na = (int64_t)K * NP + a;
                    xn[2 * na] = X;
                    xn[2 * na + 1] = Y;
                    double r = std::sqrt(X * X + Y * Y), w;
                    if (r <= cfg.r_blend0) w = 1.0;
                    else if (r >= cfg.r_blend1) w = 0.0;
                    else {
                        double z = (r - cfg.r_blend0) / (cfg.r_blend1 - cfg.r_blend0);
                        w = 1.0 - z * z * (3.0 - 2.0 * z);
                    }
                    wbl[na] = w;
                    ++a;
                }
            const double* pv[3] = { p0, p1, p2 };
            for (int f = 0; f < 3; ++f) {
                const double* u = pv[f];
                const double* v = pv[(f + 1) % 3];
                double tx = v[0] - u[0], ty = v[1] - u[1], l = std::sqrt(tx * tx + ty * ty);
                elen[3 * K + f] = l;
                enrm[6 * K + 2 * f] = ty / l;
                enrm[6 * K + 2 * f + 1] = -tx / l;
            }
            if (!cfg.wall_is_farfield)
                for (int f = 0; f < 3; ++f)
                    if (enb[3 * K + f] == -1) { wall.push_back(K); break; }
        }
        nwall = (int)wall.size();
    }

    // reference-domain coordinates of every element node [Ne][NP][2]
    void node_coords(double* xy) const override { std::memcpy(xy, xn.data(), sizeof(double) * 2 * nn); }

    // host <-> device copies are ordered on the library stream (which does not
    // synchronise with the null stream) and complete before returning
    void h2d(void* dst, const void* src, size_t bytes)
    {
        HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
    }
    void d2h(void* dst, const void* src, size_t bytes)
    {
        HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
    }

    template <class T>
    T* upload_vec(const std::vector<T>& h)
    {
        T* d = dalloc<T>((int64_t)h.size());
        h2d(d, h.data(), sizeof(T) * h.size());
        return d;
    }

    void upload()
    {
        dm.Ne = Ne;
        dm.wall_is_far = cfg.wall_is_farfield;
        dm.enb = upload_vec(enb);
        dm.etw = upload_vec(etw);
        dm.area = upload_vec(area);
        dm.jit = upload_vec(jit);
        dm.xn = upload_vec(xn);
        dm.wbl = upload_vec(wbl);
        dm.elen = upload_vec(elen);
        dm.enrm = upload_vec(enrm);
        // face tables of the stage-operator applies (one int4 per element):
        // neighbours / transposed block indices, boundary faces pointing at
        // the element itself and its own (zero) slot, bit f of .w = interior
        {
            std::vector<int4> f4(Ne), t4(Ne);
            for (int K = 0; K < Ne; ++K) {
                int nbv[3], tbv[3], mask = 0;
                for (int f = 0; f < 3; ++f) {
                    const int nb = enb[3 * K + f];
                    if (nb >= 0) {
                        mask |= 1 << f;
                        nbv[f] = nb;
                        tbv[f] = 3 * nb + etw[3 * K + f];
                    } else {
                        nbv[f] = K;
                        tbv[f] = 3 * K + f;
                    }
                }
                f4[K] = make_int4(nbv[0], nbv[1], nbv[2], mask);
                t4[K] = make_int4(tbv[0], tbv[1], tbv[2], mask);
            }
            nb4f = upload_vec(f4);
            nb4t = upload_vec(t4);
        }
        dref = dalloc<Ref<P>>(1);
        h2d(dref, &href, sizeof(Ref<P>));
        std::vector<double> mhf(NP * NP);
        for (int a = 0; a < NP; ++a)
            for (int b = 0; b < NP; ++b) mhf[a * NP + b] = href.mh[a][b];
        dmh = upload_vec(mhf);
        std::vector<int32_t> w = wall;
        if (w.empty()) w.push_back(0);
        dwall = upload_vec(w);
        dstatus = dalloc<int>(1);
        gb = dalloc<double>((nst + 1) * nn);
        dgb = dalloc<double>((nst + 1) * 3 * nn);
        tu = dalloc<double>((Nt + 1) * Nu);
        tk = dalloc<double>(nst * Nu);
        tui = dalloc<double>(nst * Nu);
        tAh = dalloc<double>(nst * 3 * Isz);
        tPd = dalloc<double>(nst * Isz);
        tAi = dalloc<double>(nst * Isz);
        Jtmp = dalloc<double>(Jsz);
        gm_b = dalloc<double>(Nu);
        gm_y = dalloc<double>(Nu);
        qh = dalloc<double>((int64_t)nst * std::max(nwall, 1) * 2);
        u0 = dalloc<double>(Nu);
        wa = dalloc<double>(Nu); wb = dalloc<double>(Nu); wc = dalloc<double>(Nu);
        wd = dalloc<double>(Nu); we = dalloc<double>(Nu); wf = dalloc<double>(Nu);
        sk3 = dalloc<double>(3 * Nu);
        fp3 = dalloc<double>(3 * Nu);
        drm = dalloc<double>(3 * Nu);
        V = dalloc<double>((int64_t)(restart + 1) * Nu);
        if (pmode != PA_PREC_FP64) {
            const int64_t n = (int64_t)nst * 3 * Isz;
            if (pmode == PA_PREC_FP32) tAl = dalloc<float>(n);
            else tAl = dalloc<bf16_t>(n);
            V32 = dalloc<float>((int64_t)(restart + 1) * Nu);
            w32 = dalloc<float>(Nu);
            r32 = dalloc<float>(Nu);
        }
        Vo = dalloc<double>((int64_t)(max_kry + 1) * Nu);
        part = dalloc<double>(mdot_blocks(Nu) * (std::max(restart, max_kry) + 2));
        hdev = dalloc<double>(std::max(restart, max_kry) + 2);
        qtmp = dalloc<double>((int64_t)std::max(nwall, 1) * 2);
        qdu = dalloc<double>((int64_t)std::max(nwall, 1) * 2 * B);
        qdmu = dalloc<double>((int64_t)std::max(nwall, 1) * 8);
        rg4 = dalloc<double>(4 * nn);
        kg4 = dalloc<double>(3 * 4 * nn);
        outer_x = dalloc<double>(Nu);
        outer_w = dalloc<double>(Nu);
        outer_z = dalloc<double>(Nu);
        outer_rhs = dalloc<double>(Nu);
        lam_buf = dalloc<double>(Nu);
        nk_delta = dalloc<double>(Nu);
        nk_save = dalloc<double>(Nu);
        gms = dalloc<GmState>(1);
        HIPCHK(hipHostMalloc((void**)&hstat, 3 * sizeof(GmHost), hipHostMallocDefault));
        use_wg = cfg.wg_solve == 1 || (cfg.wg_solve == -1 && Nu <= WG_MAXNU && restart <= WG_MAXM);
        use_graph = cfg.graph == 1;
        if (use_graph) ahp = dalloc<const double*>(1);
        if (use_wg) {
            wgst = dalloc<WgStatus>(GM_RMAX);
            HIPCHK(hipHostMalloc((void**)&hwgst, GM_RMAX * sizeof(WgStatus), hipHostMallocDefault));
        }
        for (auto& e : gm_ev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        set_jacobian_smem();
    }

    void set_jacobian_smem()
    {
        size_t smem = sizeof(JacSmem<P>);
        if (smem > 48 * 1024)
            HIPCHK(hipFuncSetAttribute((const void*)k_jacobian<P>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
    }

    // ---------------------------------------------------------------- timing
    // every TSTRIDE-th launch of a kernel is bracketed by events (an unbiased
    // sample of the launch durations with little host overhead)
    static constexpr int TSTRIDE = 8;
    int64_t tseen[PA_K_COUNT] = { 0 };
    // launches that returned at once because their GMRES system had already
    // converged (an apply enqueued ahead of the host's convergence check)
    int64_t kskip[PA_K_COUNT] = { 0 };
    void tskip(int k, int64_t n)
    {
        if (timing) kskip[k] += n;
    }
    // length-Nu vectors read or written by the working launches of the stage-
    // GMRES vector kernels: iteration j of a cycle reads j + 1 basis columns
    // and w in k_mdot_part, and also writes V_{j+1} in k_gm_upd
    int64_t kvec[PA_K_COUNT] = { 0 };
    void tvec_cycle(int64_t its)
    {
        if (!timing || its <= 0) return;
        kvec[PA_K_MDOT] += its * (its + 3) / 2;    // sum over j < its of (j + 2)
        kvec[PA_K_GMUPD] += its * (its + 5) / 2;   // sum over j < its of (j + 3)
    }
    // Every TSTRIDE-th launch of a kind (k >= 0) is sampled: its start and
    // stop events are recorded by the launch itself (hipExtLaunchKernelGGL),
    // so they bracket the kernel's execution and not the dispatch latency
    // ahead of it.  Unsampled launches are plain launches.
    bool tsample(int k, hipEvent_t* a, hipEvent_t* b)
    {
        *a = *b = nullptr;
        if (!timing || k < 0) return false;
        if ((tseen[k]++ % TSTRIDE) != 0) return false;
        if (evused >= 4096) harvest();   // every recorded pair is closed here
        if (evused == evpool.size()) {
            EvPair e;
            HIPCHK(hipEventCreate(&e.a));
            HIPCHK(hipEventCreate(&e.b));
            evpool.push_back(e);
        }
        EvPair& e = evpool[evused++];
        e.k = k;
        *a = e.a;
        *b = e.b;
        return true;
    }
    // kern<<<g, b, sm, st>>>(args...), with the kernel's start and/or stop
    // recorded into ea / eb when given
    template <class... Pm, class... Ar>
    void klaunch_ev(hipEvent_t ea, hipEvent_t eb, void (*kern)(Pm...), dim3 g, dim3 b, uint32_t sm, Ar... args)
    {
        if (ea || eb) hipExtLaunchKernelGGL(kern, g, b, sm, st, ea, eb, 0, static_cast<Pm>(args)...);
        else kern<<<g, b, sm, st>>>(static_cast<Pm>(args)...);
        LAUNCHCHK();
    }
    // the same, sampled for timing as kind k (k < 0: never)
    template <class... Pm, class... Ar>
    void klaunch(int k, void (*kern)(Pm...), dim3 g, dim3 b, uint32_t sm, Ar... args)
    {
        hipEvent_t ea, eb;
        tsample(k, &ea, &eb);
        klaunch_ev(ea, eb, kern, g, b, sm, args...);
    }
    void harvest()
    {
        if (!evused) return;
        HIPCHK(hipStreamSynchronize(st));
        for (size_t i = 0; i < evused; ++i) {
            float ms = 0;
            HIPCHK(hipEventElapsedTime(&ms, evpool[i].a, evpool[i].b));
            ktime[evpool[i].k] += ms;
            kcount[evpool[i].k] += 1;
        }
        evused = 0;
    }
    void set_timing(bool on) override
    {
        harvest();
        timing = on;
        for (int k = 0; k < PA_K_COUNT; ++k) { ktime[k] = 0; kcount[k] = 0; tseen[k] = 0; kskip[k] = 0; kvec[k] = 0; }
    }
    void kernel_time(int k, double* ms, int64_t* cnt) override
    {
        if (k < 0 || k >= PA_K_COUNT) raise(PA_EINVAL, "bad kernel id %d", k);
        // finish pending measurements without disturbing the counters
        bool t = timing;
        timing = false;
        harvest();
        timing = t;
        // sampled launches: scale the summed time to every launch seen
        double avg = kcount[k] ? ktime[k] / (double)kcount[k] : 0.0;
        if (ms) *ms = avg * (double)tseen[k];
        if (cnt) *cnt = tseen[k];
    }
    int64_t kernel_skipped(int k) override
    {
        if (k < 0 || k >= PA_K_COUNT) raise(PA_EINVAL, "bad kernel id %d", k);
        return kskip[k];
    }
    int64_t kernel_vectors(int k) override
    {
        if (k < 0 || k >= PA_K_COUNT) raise(PA_EINVAL, "bad kernel id %d", k);
        return kvec[k];
    }

    // ---------------------------------------------------------------- motion
    Motion<double> motion(double t) const
    {
        double w = 2.0 * M_PI / cfg.T;
        Motion<double> m;
        m.h = mu[0] * std::sin(w * t);
        m.hd = mu[0] * w * std::cos(w * t);
        m.th = mu[1] * std::sin(w * t + mu[2]);
        m.thd = mu[1] * w * std::cos(w * t + mu[2]);
        return m;
    }
    Motion<Dual<3>> motion_d(double t) const
    {
        double w = 2.0 * M_PI / cfg.T, s = std::sin(w * t), c = std::cos(w * t);
        double sp = std::sin(w * t + mu[2]), cp = std::cos(w * t + mu[2]);
        Motion<Dual<3>> m;
        m.h = { mu[0] * s, { s, 0, 0 } };
        m.hd = { mu[0] * w * c, { w * c, 0, 0 } };
        m.th = { mu[1] * sp, { 0, sp, mu[1] * cp } };
        m.thd = { mu[1] * w * cp, { 0, w * cp, -mu[1] * w * sp } };
        return m;
    }
    double stage_time(int n, int i) const { return n == 0 ? 0.0 : (n - 1 + rk.c[i - 1]) * dt; }
    int gidx(int n, int i) const { return n == 0 ? 0 : 1 + (n - 1) * 3 + (i - 1); }
    const double* gbs(int n, int i) const { return gb + (int64_t)gidx(n, i) * nn; }
    const double* dgbs(int n, int i) const { return dgb + (int64_t)gidx(n, i) * 3 * nn; }
    void check_stage(int n, int i) const
    {
        if (!have_params) raise(PA_ESTATE, "parameters not set");
        if (!((n == 0 && i == 0) || (n >= 1 && n <= Nt && i >= 1 && i <= 3))) raise(PA_EINVAL, "bad stage (%d,%d)", n, i);
    }

    // ---------------------------------------------------------------- kernels
    void residual(int n, int i, const double* u, double* r)
    {
        klaunch(PA_K_RESIDUAL, k_residual<P, double>, dim3(Ne), dim3(64), 0, dm, dref, ph, motion(stage_time(n, i)), u,
                gbs(n, i), nullptr, r, Nu);
    }
    void dr_dmu(int n, int i, const double* u, double* out)
    {
        k_residual<P, Dual<3>><<<Ne, 64, 0, st>>>(dm, dref, ph, motion_d(stage_time(n, i)), u, gbs(n, i), dgbs(n, i),
                                                   out, Nu);
        LAUNCHCHK();
    }
    void jacobian(int n, int i, const double* u, double* J)
    {
        klaunch(PA_K_JACOBIAN, k_jacobian<P>, dim3(Ne), dim3(320), (uint32_t)sizeof(JacSmem<P>), dm, dref, ph,
                motion(stage_time(n, i)), u, gbs(n, i), J);
    }
    // y = alpha M x + beta op(J) x
    void bsr(const double* J, double alpha, double beta, int tr, const double* x, double* y, const int* skip = nullptr)
    {
        k_bsr_apply<NP><<<Ne, 64, 0, st>>>(Ne, dm.enb, dm.etw, dm.area, dmh, J, x, y, alpha, beta, tr, skip);
        LAUNCHCHK();
    }
    // forward FP64 apply with the tile shape q (chunks per task; 0 = default)
    int fwd_q = 0;
    // (Ahp: optional device slot holding the operator's address, read by
    // the kernel; k: timing kind, < 0 for none)
    void launch_fwd(int q, const double* Ah, const double* x, double* y, const int* skip,
                    const double* const* Ahp = nullptr, int k = -1)
    {
        const dim3 g(Ne), b(64);
        if (q == 1 && ahat_fwd_valid<NP, double>(1))
            klaunch(k, k_ahat_fwd<NP, double, double, 1>, g, b, 0, Ne, nb4f, Ah, x, y, skip, Ahp);
        else if (q == 2 && ahat_fwd_valid<NP, double>(2))
            klaunch(k, k_ahat_fwd<NP, double, double, 2>, g, b, 0, Ne, nb4f, Ah, x, y, skip, Ahp);
        else if (q == 4 && ahat_fwd_valid<NP, double>(4)) {
            if constexpr (ahat_fwd_valid<NP, double>(4))
                klaunch(k, k_ahat_fwd<NP, double, double, 4>, g, b, 0, Ne, nb4f, Ah, x, y, skip, Ahp);
        } else
            klaunch(k, k_ahat_fwd<NP, double, double>, g, b, 0, Ne, nb4f, Ah, x, y, skip, Ahp);
    }
    // autotune (pa_config.autotune): time each valid tile shape on the first
    // stored stage operator (after its formation, 10 launches each, HIP
    // events, scratch vectors of its own) and keep the fastest.  Off by
    // default: the shape fixes the summation order, so a timing-dependent
    // choice would make otherwise identical runs differ in the last bits.
    bool fwd_tuned = false;
    double fwd_tune_us[3] = { 0, 0, 0 };
    double *tune_x = nullptr, *tune_y = nullptr;
    void tune_fwd(const double* Ah)
    {
        fwd_tuned = true;
        if (!tune_x) {
            tune_x = dalloc<double>(Nu);
            tune_y = dalloc<double>(Nu);
            zero(tune_x);
        }
        const int qs[3] = { 1, 2, 4 };
        hipEvent_t a, b;
        HIPCHK(hipEventCreate(&a));
        HIPCHK(hipEventCreate(&b));
        double best = 1e300;
        for (int k = 0; k < 3; ++k) {
            const int q = qs[k];
            const bool ok = q == 1 ? ahat_fwd_valid<NP, double>(1)
                            : q == 2 ? ahat_fwd_valid<NP, double>(2) : ahat_fwd_valid<NP, double>(4);
            if (!ok) { fwd_tune_us[k] = -1; continue; }
            launch_fwd(q, Ah, tune_x, tune_y, nullptr);   // warm
            HIPCHK(hipEventRecord(a, st));
            for (int r = 0; r < 10; ++r) launch_fwd(q, Ah, tune_x, tune_y, nullptr);
            HIPCHK(hipEventRecord(b, st));
            HIPCHK(hipEventSynchronize(b));
            float ms = 0;
            HIPCHK(hipEventElapsedTime(&ms, a, b));
            fwd_tune_us[k] = ms * 100.0;   // us per launch
            if (fwd_tune_us[k] < best) { best = fwd_tune_us[k]; fwd_q = q; }
        }
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        if (verbose)
            fprintf(stderr, "[pa] forward apply tiles: 1/2/4 chunks per task %.1f/%.1f/%.1f us -> %d\n",
                    fwd_tune_us[0], fwd_tune_us[1], fwd_tune_us[2], fwd_q);
    }
    void ahat(const double* Ah, int tr, const double* x, double* y, const int* skip = nullptr)
    {
        const double* const* noslot = nullptr;
        if (tr) klaunch(PA_K_SPMV_T, k_ahat_tr<NP, double, double>, dim3(Ne), dim3(64), 0, Ne, nb4t, Ah, x, y, skip, noslot);
        else launch_fwd(fwd_q, Ah, x, y, skip, nullptr, PA_K_SPMV);
    }
    void ahat_lo(const void* Al, int tr, const float* x, float* y, const int* skip = nullptr)
    {
        const int k = PA_K_SPMV_LO;
        const dim3 g(Ne), b(64);
        const float* const* nof = nullptr;
        const bf16_t* const* nob = nullptr;
        if (tr) {
            if (pmode == PA_PREC_FP32)
                klaunch(k, k_ahat_tr<NP, float, float>, g, b, 0, Ne, nb4t, (const float*)Al, x, y, skip, nof);
            else if constexpr (B % 8 == 0)
                klaunch(k, k_ahat_tr<NP, bf16_t, float>, g, b, 0, Ne, nb4t, (const bf16_t*)Al, x, y, skip, nob);
            else   // 16-byte BF16 chunks would straddle rows
                klaunch(k, k_ahat_apply_lo<NP, bf16_t>, g, b, 0, Ne, dm.enb, dm.etw, (const bf16_t*)Al, x, y, tr, skip);
        } else {
            if (pmode == PA_PREC_FP32)
                klaunch(k, k_ahat_fwd<NP, float, float>, g, b, 0, Ne, nb4f, (const float*)Al, x, y, skip, nof);
            else if constexpr (B % 8 == 0)
                klaunch(k, k_ahat_fwd<NP, bf16_t, float>, g, b, 0, Ne, nb4f, (const bf16_t*)Al, x, y, skip, nob);
            else   // 16-byte BF16 chunks would straddle rows
                klaunch(k, k_ahat_apply_lo<NP, bf16_t>, g, b, 0, Ne, dm.enb, dm.etw, (const bf16_t*)Al, x, y, tr, skip);
        }
    }
    void prec(const double* Ai, int tr, const double* x, double* z, const int* skip = nullptr)
    {
        klaunch(PA_K_PRECOND, k_block_apply<NP>, dim3(Ne), dim3(64), 0, Ne, Ai, x, z, tr, skip);
    }
    void axpby(double a, const double* x, double b, double* y)
    {
        k_axpby<<<grid1(Nu), 256, 0, st>>>(a, x, b, y, Nu);
        LAUNCHCHK();
    }
    void lincomb(double a, const double* x, double b, const double* y, double* z)
    {
        k_lincomb<<<grid1(Nu), 256, 0, st>>>(a, x, b, y, z, Nu);
        LAUNCHCHK();
    }
    void copy(const double* x, double* y)
    {
        HIPCHK(hipMemcpyAsync(y, x, sizeof(double) * Nu, hipMemcpyDeviceToDevice, st));
    }
    void zero(double* y, int64_t n = -1)
    {
        HIPCHK(hipMemsetAsync(y, 0, sizeof(double) * (n < 0 ? Nu : n), st));
    }
    // host h[c] = <V_c, w>, c < ncols (V_c = V + c*ldv); one synchronisation
    void dots(const double* Vb, int64_t ldv, int ncols, const double* w, double* h)
    {
        const int nb = (int)mdot_blocks(Nu);
        k_mdot_part<<<dim3(nb, mdot_chunks(ncols)), MD_THREADS, 0, st>>>(Vb, ldv, ncols, 0, w, Nu, part, nullptr);
        k_mdot_fin<<<1, MD_THREADS, 0, st>>>(part, nb, ncols, hdev);
        LAUNCHCHK();
        HIPCHK(hipMemcpyAsync(h, hdev, sizeof(double) * ncols, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
    }
    double norm(const double* w)
    {
        double h;
        dots(w, 0, 1, w, &h);
        return std::sqrt(h);
    }
    // w += sign * sum_c h[c] V_c  (h host)
    void vupdate(const double* Vb, int64_t ldv, int ncols, const double* h, double sign, double* w)
    {
        HIPCHK(hipMemcpyAsync(hdev, h, sizeof(double) * ncols, hipMemcpyHostToDevice, st));
        k_vupdate<<<grid1(Nu), 256, 0, st>>>(Vb, ldv, ncols, hdev, sign, w, Nu);
        LAUNCHCHK();
    }

    // ---------------------------------------------------------------- GMRES
    // Generic GMRES (Arnoldi with classical Gram-Schmidt and one
    // reorthogonalisation, Givens rotations, zero initial guess).
    // A(v, out), Pc(v, out) or empty for no preconditioner (right
    // preconditioning).  Basis storage Vb with room for m+1 vectors.
    // Returns iterations; throws PA_ENOCONV when maxit is reached and
    // require_conv is set.
    int gmres(const std::function<void(const double*, double*)>& A,
              const std::function<void(const double*, double*)>& Pc, const double* b, double* x, double rtol,
              int m, int maxit, double* Vb, double* wk, double* zk, double* relres, bool require_conv)
    {
        std::vector<double> H((m + 1) * m, 0.0), cs(m), sn(m), g(m + 1), y(m), h(m + 2), h2(m + 2);
        double bn = norm(b);
        zero(x);
        if (relres) *relres = 0.0;
        if (bn == 0.0) return 0;
        int total = 0;
        bool first = true;
        double res = bn;
        for (;;) {
            // r = b - A x
            if (first) copy(b, wk);
            else { A(x, wk); lincomb(1.0, b, -1.0, wk, wk); }
            double beta = first ? bn : norm(wk);
            first = false;
            res = beta;
            if (beta <= rtol * bn) break;
            if (total >= maxit) break;
            lincomb(1.0 / beta, wk, 0.0, wk, Vb);
            std::fill(g.begin(), g.end(), 0.0);
            g[0] = beta;
            int j = 0;
            bool done = false;
            for (; j < m && total < maxit; ++j) {
                ++total;
                double* vj = Vb + (int64_t)j * Nu;
                if (Pc) { Pc(vj, zk); A(zk, wk); } else A(vj, wk);
                dots(Vb, Nu, j + 1, wk, h.data());
                vupdate(Vb, Nu, j + 1, h.data(), -1.0, wk);
                // second pass; the last column returns |w|^2 for the norm
                {
                    const int nb = (int)mdot_blocks(Nu);
                    k_mdot_part<<<dim3(nb, mdot_chunks(j + 2)), MD_THREADS, 0, st>>>(Vb, Nu, j + 1, 1, wk, Nu, part, nullptr);
                    k_mdot_fin<<<1, MD_THREADS, 0, st>>>(part, nb, j + 2, hdev);
                    LAUNCHCHK();
                    HIPCHK(hipMemcpyAsync(h2.data(), hdev, sizeof(double) * (j + 2), hipMemcpyDeviceToHost, st));
                    HIPCHK(hipStreamSynchronize(st));
                }
                double ww = h2[j + 1], corr = 0.0;
                for (int i = 0; i <= j; ++i) corr += h2[i] * h2[i];
                vupdate(Vb, Nu, j + 1, h2.data(), -1.0, wk);
                for (int i = 0; i <= j; ++i) H[i * m + j] = h[i] + h2[i];
                double hn = std::sqrt(std::max(ww - corr, 0.0));
                if (!std::isfinite(hn)) raise(PA_ENUMERIC, "NaN in GMRES");
                H[(j + 1) * m + j] = hn;
                for (int i = 0; i < j; ++i) {
                    double a = H[i * m + j], bb = H[(i + 1) * m + j];
                    H[i * m + j] = cs[i] * a + sn[i] * bb;
                    H[(i + 1) * m + j] = -sn[i] * a + cs[i] * bb;
                }
                double a = H[j * m + j], bb = H[(j + 1) * m + j];
                double rr = std::sqrt(a * a + bb * bb);
                cs[j] = a / rr;
                sn[j] = bb / rr;
                H[j * m + j] = rr;
                H[(j + 1) * m + j] = 0.0;
                g[j + 1] = -sn[j] * g[j];
                g[j] = cs[j] * g[j];
                res = std::fabs(g[j + 1]);
                if (res <= rtol * bn || hn == 0.0) { ++j; done = true; break; }
                lincomb(1.0 / hn, wk, 0.0, wk, Vb + (int64_t)(j + 1) * Nu);
            }
            for (int i = j - 1; i >= 0; --i) {
                double s = g[i];
                for (int k = i + 1; k < j; ++k) s -= H[i * m + k] * y[k];
                y[i] = s / H[i * m + i];
            }
            zero(wk);
            vupdate(Vb, Nu, j, y.data(), 1.0, wk);
            if (Pc) { Pc(wk, zk); axpby(1.0, zk, 1.0, x); }
            else axpby(1.0, wk, 1.0, x);
            if (done) break;
        }
        if (relres) *relres = res / bn;
        if (res > rtol * bn && require_conv) raise(PA_ENOCONV, "GMRES did not converge: rel. residual %.3e", res / bn);
        return total;
    }

    // stage solve: (M - c J) x = rhs, or its transpose, with the stored
    // block-Jacobi inverse Ai
    // Stage solve with the block-Jacobi factor folded into Ahat = A P^{-1}:
    //   forward:    Ahat y = rhs,          x = P^{-1} y   (right preconditioning)
    //   transposed: Ahat^T x = P^{-T} rhs                 (left preconditioning)
    // GMRES(m) with the Arnoldi state on the device: no host round trip
    // inside an iteration.  Every GM_CHECK iterations the status is copied
    // to pinned memory behind an event; the host waits for the previous
    // copy only, so GM_CHECK iterations stay queued on the device while it
    // looks.  Iterations enqueued after convergence exit at once.
    static constexpr int GM_CHECK = 5;

    // pa_config.graph: the GM_CHECK iterations between two checks (apply,
    // multi-dot, update; one system or R sharing the operator), for one
    // transpose flag, system count and first column, are captured on the
    // stream once and replayed.  Every launch of such a graph names the
    // context's own fixed buffers (basis, work vector, partial sums, GMRES
    // states); only the stage operator changes between solves, and the
    // applies read its address from the device slot ahp, set on the stream
    // before each solve.  A replay runs the kernels a host loop would
    // launch, with the same arguments, in the same order.
    bool use_graph = false;
    const double** ahp = nullptr;
    hipGraphExec_t gx[2][GM_RMAX + 1][GM_MAXM / GM_CHECK] = {};
    int gx_q = -1;   // forward tile shape the graphs were captured with
    void set_graph_op(const double* Ah)
    {
        k_set_ptr<<<1, 64, 0, st>>>(ahp, Ah);
        LAUNCHCHK();
    }
    void free_graphs()
    {
        for (auto& a : gx)
            for (auto& b : a)
                for (auto& g : b)
                    if (g) {
                        (void)hipGraphExecDestroy(g);
                        g = nullptr;
                    }
    }
    // iteration j of the stage solve (R == 1: the buffers of stage_solve;
    // R > 1: those of stage_solve_multi), with the operator from the slot
    void gm_iter_slot(int tr, int R, int j)
    {
        const int m = restart, nb = (int)mdot_blocks(Nu);
        if (R == 1) {
            const double* vj = V + (int64_t)j * Nu;
            if (tr) k_ahat_tr<NP, double, double><<<Ne, 64, 0, st>>>(Ne, nb4t, nullptr, vj, we, &gms->done, ahp);
            else launch_fwd(fwd_q, nullptr, vj, we, &gms->done, ahp);
            k_mdot_part<<<dim3(nb, mdot_chunks(j + 2)), MD_THREADS, 0, st>>>(V, Nu, j + 1, 1, we, Nu, part, gms);
            k_gm_upd<<<(unsigned)gm_upd_blocks(Nu), GU_THREADS, 0, st>>>(V, Nu, j, m, we, Nu, part, nb, gms);
        } else {
            const int64_t sV = (int64_t)(m + 1) * Nu, sP = (int64_t)nb * (m + 2);
            ahat_m(nullptr, tr, R, Vm + (int64_t)j * Nu, sV, wm, Nu, gmsm, ahp);
            k_mdot_part<<<dim3(nb, mdot_chunks(j + 2) * R), MD_THREADS, 0, st>>>(Vm, Nu, j + 1, 1, wm, Nu, partm,
                                                                                 gmsm, sV, Nu, sP);
            k_gm_upd<<<dim3((unsigned)gm_upd_blocks(Nu), R), GU_THREADS, 0, st>>>(Vm, Nu, j, m, wm, Nu, partm, nb,
                                                                                  gmsm, sV, Nu, sP);
        }
    }
    // the graph of iterations c GM_CHECK .. (c + 1) GM_CHECK - 1, captured on first use
    hipGraphExec_t gm_graph(int tr, int R, int c)
    {
        if (gx_q != fwd_q) {
            free_graphs();
            gx_q = fwd_q;
        }
        hipGraphExec_t& g = gx[tr][R][c];
        if (g) return g;
        (void)hipGetLastError();
        HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        hipGraph_t gr = nullptr;
        try {
            for (int j = c * GM_CHECK; j < (c + 1) * GM_CHECK; ++j) gm_iter_slot(tr, R, j);
        } catch (...) {   // leave the stream out of capture mode
            if (hipStreamEndCapture(st, &gr) == hipSuccess && gr) (void)hipGraphDestroy(gr);
            throw;
        }
        const hipError_t el = hipGetLastError();
        const hipError_t ec = hipStreamEndCapture(st, &gr);
        if (el != hipSuccess || ec != hipSuccess || !gr) {
            if (gr) (void)hipGraphDestroy(gr);
            raise(PA_EDEVICE, "stage-GMRES graph capture failed: %s",
                  hipGetErrorString(el != hipSuccess ? el : ec));
        }
        const hipError_t ei = hipGraphInstantiate(&g, gr, nullptr, nullptr, 0);
        (void)hipGraphDestroy(gr);
        if (ei != hipSuccess) {
            g = nullptr;
            raise(PA_EDEVICE, "stage-GMRES graph instantiation failed: %s", hipGetErrorString(ei));
        }
        return g;
    }
    // R systems sharing one stage operator, each solved by one workgroup
    // (k_stage_gmres_wg): rhs and x hold R vectors; returns the largest
    // iteration count
    int stage_solve_wg(const StageOps& op, int tr, int R, const double* rhs, double* x, double* Vb, double* yb,
                       double* wb)
    {
        const int m = restart, maxit = 20 * restart;
        const double* b = rhs;
        if (tr) {
            double* bt = R == 1 ? gm_b : bm;
            for (int r = 0; r < R; ++r) prec(op.Pinv, 1, rhs + r * Nu, bt + r * Nu);
            b = bt;
        }
        k_stage_gmres_wg<NP><<<R, WG_THREADS, 0, st>>>(Ne, dm.enb, dm.etw, op.Ah, tr, b, yb, Vb, wb, m, maxit,
                                                        cfg.lin_rtol, wgst, Nu, Nu, (int64_t)(m + 1) * Nu, Nu);
        LAUNCHCHK();
        HIPCHK(hipMemcpyAsync(hwgst, wgst, R * sizeof(WgStatus), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        int its = 0;
        for (int r = 0; r < R; ++r) {
            if (hwgst[r].conv < 0) raise(PA_ENUMERIC, "NaN in stage GMRES");
            if (hwgst[r].conv == 0)
                raise(PA_ENOCONV, "stage GMRES did not converge in %d iterations: residual %.3e", hwgst[r].its,
                      hwgst[r].res);
            its = std::max(its, hwgst[r].its);
            cnt_gmres += hwgst[r].its;
        }
        for (int r = 0; r < R; ++r) {
            if (tr) copy(yb + r * Nu, x + r * Nu);
            else prec(op.Pinv, 0, yb + r * Nu, x + r * Nu);
        }
        return its;
    }
    // x0 (optional, may alias x): initial guess in the stage unknowns; it is
    // used when its residual is below |b|, else the solve starts from zero.
    // The stopping test stays relative to |b|.
    int stage_solve(const StageOps& op, int tr, const double* rhs, double* x, const double* x0 = nullptr)
    {
        if (pmode != PA_PREC_FP64) return stage_solve_ir(op, tr, rhs, x);
        if (use_wg) return stage_solve_wg(op, tr, 1, rhs, x, V, gm_y, we);
        const int m = restart, maxit = 20 * restart;
        const int* skip = &gms->done;
        const int nb = (int)mdot_blocks(Nu);
        const double* b = rhs;
        if (tr) { prec(op.Pinv, 1, rhs, gm_b); b = gm_b; }
        const double bn = norm(b);
        if (bn == 0.0) { zero(x); return 0; }
        const double tol = cfg.lin_rtol * bn;
        double* r = we;
        double* w = we;
        double* y = gm_y;
        int total = 0;
        bool guessed = false;
        if (x0) {   // y0 = P x0 (forward) or x0 (transposed), r0 = b - Ahat y0
            if (tr) copy(x0, y);
            else prec(op.Pd, 0, x0, y);
            ahat(op.Ah, tr, y, w);
            lincomb(1.0, b, -1.0, w, r);
            guessed = norm(r) < bn;
            ++cnt_guess_try;
            if (guessed) ++cnt_guess_used;
        }
        if (!guessed) {
            zero(y);
            copy(b, r);
        }
        if (use_graph) set_graph_op(op.Ah);
        for (;;) {
            k_mdot_part<<<nb, MD_THREADS, 0, st>>>(r, 0, 1, 0, r, Nu, part, nullptr);
            k_gm_begin<<<nb, MD_THREADS, 0, st>>>(r, V, Nu, part, nb, GmTol{ { tol } }, gms);
            LAUNCHCHK();
            int pending = -1, slot = 0, launched = 0;
            for (int j = 0; j < m; ++j) {
                if (use_graph) {
                    // iterations j .. j + GM_CHECK - 1 (m is a multiple of GM_CHECK)
                    if (j % GM_CHECK == 0) HIPCHK(hipGraphLaunch(gm_graph(tr, 1, j / GM_CHECK), st));
                } else {
                    double* vj = V + (int64_t)j * Nu;
                    ahat(op.Ah, tr, vj, w, skip);
                    // one classical Gram-Schmidt pass; the cycle closes on cancellation
                    klaunch(PA_K_MDOT, k_mdot_part<double>, dim3(nb, mdot_chunks(j + 2)), dim3(MD_THREADS), 0, V, Nu,
                            j + 1, 1, w, Nu, part, gms, 0, 0, 0);
                    klaunch(PA_K_GMUPD, k_gm_upd<double>, dim3((unsigned)gm_upd_blocks(Nu)), dim3(GU_THREADS), 0, V,
                            Nu, j, m, w, Nu, part, nb, gms, 0, 0, 0);
                }
                ++launched;
                if ((j + 1) % GM_CHECK == 0 && j < m - 1) {
                    if (pending >= 0) {
                        HIPCHK(hipEventSynchronize(gm_ev[pending]));
                        if (hstat[pending].done) break;
                    }
                    HIPCHK(hipMemcpyAsync(&hstat[slot], &gms->res, sizeof(GmHost), hipMemcpyDeviceToHost, st));
                    HIPCHK(hipEventRecord(gm_ev[slot], st));
                    pending = slot;
                    slot ^= 1;
                }
            }
            HIPCHK(hipMemcpyAsync(&hstat[2], &gms->res, sizeof(GmHost), hipMemcpyDeviceToHost, st));
            // y += V ycoef
            k_gm_solve<<<1, 256, 0, st>>>(m, gms);
            k_gm_combine<<<grid1(Nu), 256, 0, st>>>(V, Nu, m, w, Nu, gms);
            LAUNCHCHK();
            axpby(1.0, w, 1.0, y);
            // true residual r = b - Ahat y: accepts a converged cycle (the
            // Arnoldi estimate can drift when Gram-Schmidt skips its second
            // pass) or restarts the next one
            ahat(op.Ah, tr, y, w);
            lincomb(1.0, b, -1.0, w, r);
            const double rn = norm(r);   // synchronises: hstat[2] is valid below
            const bool done = hstat[2].done != 0;
            total += done ? hstat[2].its : m;
            tskip(tr ? PA_K_SPMV_T : PA_K_SPMV, launched - (done ? hstat[2].its : m));
            tskip(PA_K_MDOT, launched - (done ? hstat[2].its : m));
            tskip(PA_K_GMUPD, launched - (done ? hstat[2].its : m));
            tvec_cycle(done ? hstat[2].its : m);
            if (done && !std::isfinite(hstat[2].res)) raise(PA_ENUMERIC, "NaN in stage GMRES");
            if (!std::isfinite(rn)) raise(PA_ENUMERIC, "NaN in stage GMRES");
            if (done && rn <= 2.0 * tol) break;
            if (total >= maxit)
                raise(PA_ENOCONV, "stage GMRES did not converge in %d iterations: rel. residual %.3e", total,
                      rn / bn);
        }
        if (tr) copy(y, x);
        else prec(op.Pinv, 0, y, x);
        cnt_gmres += total;
        return total;
    }
    // Mixed-precision stage solve by iterative refinement on the same
    // preconditioned system as stage_solve (forward: Ahat y = b, x = P^{-1} y;
    // transposed: Ahat^T x = P^{-T} b).  The residual r = b - Ahat y, the
    // update y += |r| d and the stopping test |r| <= lin_rtol |b| are FP64;
    // each correction d is one GMRES cycle in FP32 on Ahat_lo d = r / |r|,
    // stopped at the relative reduction the stored precision can still
    // deliver (FP32 1e-6, BF16 1e-2) or at the tolerance, whichever is larger.
    int stage_solve_ir(const StageOps& op, int tr, const double* rhs, double* x)
    {
        const int m = restart, maxit = 20 * restart;
        const int* skip = &gms->done;
        const int nb = (int)mdot_blocks(Nu);
        const double floor_red = pmode == PA_PREC_FP32 ? 1e-6 : 1e-2;
        const double* b = rhs;
        if (tr) { prec(op.Pinv, 1, rhs, gm_b); b = gm_b; }
        const double bn = norm(b);
        zero(x);
        if (bn == 0.0) return 0;
        const double tol = cfg.lin_rtol * bn;
        double* r = we;
        double* y = gm_y;
        zero(y);
        copy(b, r);
        double rn = bn;
        int total = 0;
        for (;;) {
            k_scale_to_f32<<<grid1(Nu), 256, 0, st>>>(1.0 / rn, r, r32, Nu);
            k_mdot_part<<<nb, MD_THREADS, 0, st>>>(r32, 0, 1, 0, r32, Nu, part, nullptr);
            k_gm_begin<<<nb, MD_THREADS, 0, st>>>(r32, V32, Nu, part, nb, GmTol{ { std::max(tol / rn, floor_red) } },
                                                  gms);
            LAUNCHCHK();
            int pending = -1, slot = 0, launched = 0;
            for (int j = 0; j < m; ++j) {
                float* vj = V32 + (int64_t)j * Nu;
                ahat_lo(op.Al, tr, vj, w32, skip);
                ++launched;
                k_mdot_part<<<dim3(nb, mdot_chunks(j + 2)), MD_THREADS, 0, st>>>((const float*)V32, Nu, j + 1, 1,
                                                                                  (const float*)w32, Nu, part, gms);
                k_gm_upd<<<(unsigned)gm_upd_blocks(Nu), GU_THREADS, 0, st>>>((const float*)V32, Nu, j, m,
                                                                             (const float*)w32, Nu, part, nb, gms);
                LAUNCHCHK();
                if ((j + 1) % GM_CHECK == 0 && j < m - 1) {
                    if (pending >= 0) {
                        HIPCHK(hipEventSynchronize(gm_ev[pending]));
                        if (hstat[pending].done) break;
                    }
                    HIPCHK(hipMemcpyAsync(&hstat[slot], &gms->res, sizeof(GmHost), hipMemcpyDeviceToHost, st));
                    HIPCHK(hipEventRecord(gm_ev[slot], st));
                    pending = slot;
                    slot ^= 1;
                }
            }
            HIPCHK(hipMemcpyAsync(&hstat[2], &gms->res, sizeof(GmHost), hipMemcpyDeviceToHost, st));
            k_gm_solve<<<1, 256, 0, st>>>(m, gms);
            k_gm_combine<<<grid1(Nu), 256, 0, st>>>((const float*)V32, Nu, m, r, Nu, gms);
            LAUNCHCHK();
            axpby(rn, r, 1.0, y);
            // FP64 refinement residual
            ahat(op.Ah, tr, y, r);
            lincomb(1.0, b, -1.0, r, r);
            rn = norm(r);   // synchronises: hstat[2] is valid below
            total += hstat[2].done ? hstat[2].its : m;
            tskip(PA_K_SPMV_LO, launched - (hstat[2].done ? hstat[2].its : m));
            if (!std::isfinite(rn) || !std::isfinite(hstat[2].res)) raise(PA_ENUMERIC, "NaN in stage GMRES");
            if (rn <= tol) break;
            if (total >= maxit)
                raise(PA_ENOCONV, "stage GMRES (mixed precision) did not converge in %d iterations: rel. residual %.3e",
                      total, rn / bn);
        }
        if (tr) copy(y, x);
        else prec(op.Pinv, 0, y, x);
        cnt_gmres += total;
        return total;
    }
    // ---------------------------------------------------------------- learned warm start
    // POD of method-generated periodic initial states (snapshot method: the
    // Gram matrix of the centred states on the device, its eigenpairs on
    // the host, the modes formed on the device) and an MLP from normalised
    // parameters to normalised POD coefficients, trained with Adam.
    Mlp mlp;
    int ws_k = 0;
    double *ws_mean = nullptr, *ws_psi = nullptr;
    float* ws_cs = nullptr;                   // device coefficient scales [ws_k]
    std::vector<float> ws_cs_h;
    // perceptron inputs (h0, theta0, phi, Mach): normalisation offsets and scales
    static constexpr int WS_NIN = 4;
    float ws_xm[WS_NIN] = { 0, 0, 0, 0 }, ws_xs[WS_NIN] = { 1, 1, 1, 1 };
    std::vector<double> ws_lam;               // Gram-matrix eigenvalues of the kept modes
    static constexpr int WS_MAXK = 128;
    // free stream gbar(0; m) U_inf(mach) at t = 0 for kinematics m, into out [Nu]
    void freestream_for(const double m[3], double mach, double* out)
    {
        Motion<double> mo;
        const double w = 2.0 * M_PI / cfg.T;
        mo.h = 0.0;
        mo.hd = m[0] * w;
        mo.th = m[1] * std::sin(m[2]);
        mo.thd = m[1] * w * std::cos(m[2]);
        k_gbar0<P, double><<<Ne, 64, 0, st>>>(dm, dref, mo, rg4, nn);
        LAUNCHCHK();
        const double pinf = 1.0 / (cfg.gamma * mach * mach);
        const double4 Ui{ 1.0, 1.0, 0.0, pinf / (cfg.gamma - 1.0) + 0.5 };
        k_scale_state<<<grid1(nn), 256, 0, st>>>(rg4, Ui, out, nn);
        LAUNCHCHK();
    }
    void ws_alloc()
    {
        if (ws_mean) return;
        ws_mean = dalloc<double>(Nu);
        ws_psi = dalloc<double>((int64_t)WS_MAXK * Nu);
        ws_cs = dalloc<float>(WS_MAXK);
    }
    void ws_train(const double* params, const double* states, int S, const pa_ws_opts& o, double* final_loss) override
    {
        if (S < 2 || !params || !states) raise(PA_EINVAL, "need at least two training states");
        if (o.modes < 1 || o.width < 1 || o.epochs < 0 || !(o.lr > 0)) raise(PA_EINVAL, "bad warm-start options");
        ws_alloc();
        double* D = static_cast<double*>(da.get(sizeof(double) * (size_t)S * Nu));
        struct Free { const DevAlloc& a; double* q; ~Free() { a.put(q); } } fd{ da, D };
        h2d(D, states, sizeof(double) * (size_t)S * Nu);
        // deviation of each snapshot from the free stream of its own
        // kinematics and Mach number, then mean and centred snapshots
        for (int i = 0; i < S; ++i) {
            const double* pm = params + (size_t)WS_NIN * i;
            if (!(pm[3] > 0.0)) raise(PA_EINVAL, "training Mach number must be positive");
            freestream_for(pm, pm[3], wf);
            axpby(-1.0, wf, 1.0, D + (int64_t)i * Nu);
        }
        zero(ws_mean);
        for (int i = 0; i < S; ++i) axpby(1.0 / S, D + (int64_t)i * Nu, 1.0, ws_mean);
        for (int i = 0; i < S; ++i) axpby(-1.0, ws_mean, 1.0, D + (int64_t)i * Nu);
        std::vector<double> G((size_t)S * S), row(S);
        for (int i = 0; i < S; ++i) {
            dots(D, Nu, i + 1, D + (int64_t)i * Nu, row.data());
            for (int j = 0; j <= i; ++j) G[(size_t)i * S + j] = G[(size_t)j * S + i] = row[j];
        }
        std::vector<double> lam, Vg;
        sym_eig(G, S, lam, Vg);
        int k = std::min({ o.modes, S - 1, WS_MAXK });
        while (k > 1 && !(lam[k - 1] > 1e-13 * lam[0])) --k;
        if (!(lam[0] > 0.0)) raise(PA_EINVAL, "training states are all equal");
        ws_k = k;
        ws_lam.assign(lam.begin(), lam.begin() + k);
        ws_cs_h.assign(k, 0.0f);
        std::vector<double> coef(S);
        std::vector<float> Th((size_t)k * S);
        for (int j = 0; j < k; ++j) {
            const double sl = std::sqrt(lam[j]);
            for (int i = 0; i < S; ++i) coef[i] = Vg[(size_t)i * S + j] / sl;
            zero(ws_psi + (int64_t)j * Nu);
            vupdate(D, Nu, S, coef.data(), 1.0, ws_psi + (int64_t)j * Nu);
            // coefficients of the training states: c_j,i = sqrt(lam_j) V[i][j];
            // scaled by their RMS sqrt(lam_j / S)
            ws_cs_h[j] = (float)std::sqrt(lam[j] / S);
            for (int i = 0; i < S; ++i) Th[(size_t)j * S + i] = (float)(std::sqrt((double)S) * Vg[(size_t)i * S + j]);
        }
        h2d(ws_cs, ws_cs_h.data(), sizeof(float) * k);
        // normalised inputs
        std::vector<float> Xh((size_t)WS_NIN * S);
        for (int c = 0; c < WS_NIN; ++c) {
            double mean = 0, var = 0;
            for (int i = 0; i < S; ++i) mean += params[WS_NIN * i + c];
            mean /= S;
            for (int i = 0; i < S; ++i) var += (params[WS_NIN * i + c] - mean) * (params[WS_NIN * i + c] - mean);
            const double sd = std::sqrt(var / S);
            ws_xm[c] = (float)mean;
            ws_xs[c] = (float)(sd > 1e-12 ? sd : 1.0);
            for (int i = 0; i < S; ++i) Xh[(size_t)c * S + i] = (float)((params[WS_NIN * i + c] - mean) / ws_xs[c]);
        }
        mlp.init(WS_NIN, o.width, k, st);
        std::vector<float> P0(mlp.nparam, 0.0f);
        uint64_t sd = o.seed;
        for (int l = 0; l < 4; ++l) {
            const int fi = mlp.sh.dims[l], fo = mlp.sh.dims[l + 1];
            const double a = std::sqrt(6.0 / (fi + fo));
            for (int64_t q = 0; q < (int64_t)fi * fo; ++q) {
                const double u = (double)(splitmix64(sd) >> 11) * (1.0 / 9007199254740992.0);
                P0[mlp.sh.woff[l] + q] = (float)((2.0 * u - 1.0) * a);
            }
        }
        h2d(mlp.p, P0.data(), sizeof(float) * mlp.nparam);
        mlp.reserve(S);
        h2d(mlp.X, Xh.data(), sizeof(float) * Xh.size());
        h2d(mlp.T, Th.data(), sizeof(float) * Th.size());
        for (int e = 0; e < o.epochs; ++e) {
            mlp.forward(S);
            mlp.mse(S);
            mlp.backward(S);
            mlp.adam(o.lr);
        }
        mlp.forward(S);
        mlp.mse(S);
        float L = 0;
        d2h(&L, mlp.loss, sizeof(float));
        if (final_loss) *final_loss = L;
        if (verbose) fprintf(stderr, "[pa] warm start: %d states, %d modes, %d epochs, loss %.3e\n", S, k, o.epochs, L);
    }
    void ws_predict(const double m[3]) override
    {
        if (!ws_k) raise(PA_ESTATE, "no trained warm-start model");
        // inputs: the kinematics and this context's Mach number
        const double in[WS_NIN] = { m[0], m[1], m[2], cfg.mach };
        float x[WS_NIN];
        for (int c = 0; c < WS_NIN; ++c) x[c] = (float)((in[c] - ws_xm[c]) / ws_xs[c]);
        mlp.reserve(1);
        // a single column: X [WS_NIN][1]
        h2d(mlp.X, x, sizeof x);
        mlp.forward(1);
        // u0 = free stream + mean deviation + modes x coefficients
        freestream_for(m, cfg.mach, wf);
        axpby(1.0, ws_mean, 1.0, wf);
        k_pod_expand<<<grid1(Nu), 256, 0, st>>>(wf, ws_psi, ws_k, Nu, mlp.out(), ws_cs, u0, Nu);
        LAUNCHCHK();
        HIPCHK(hipStreamSynchronize(st));
        have_traj = false;
    }
    // shooting from the predicted state; if the first Newton step does not
    // lower ||R|| (or fails), start again from the free stream
    void ws_shoot(double tol, double eta, int maxit, pa_shoot_report* rep, int32_t* fell_back) override
    {
        if (!have_params) raise(PA_ESTATE, "set the parameters first");
        ws_predict(mu);
        pa_shoot_report r1{}, r2{};
        if (rep) {   // the history describes the last shooting run
            for (pa_shoot_report* q : { &r1, &r2 }) {
                q->res_hist = rep->res_hist;
                q->krylov_hist = rep->krylov_hist;
                q->step_hist = rep->step_hist;
                q->hist_cap = rep->hist_cap;
            }
        }
        bool progressed = false, converged = false;
        try {
            shoot(tol, eta, 1, &r1);
            converged = true;
        } catch (const PaError& e) {
            if (e.code != PA_ENOCONV && e.code != PA_ENUMERIC) throw;
            progressed = r1.newton_its >= 1 && r1.res < r1.res0;
        }
        if (fell_back) *fell_back = 0;
        if (!converged) {
            if (progressed) {
                shoot(tol, eta, std::max(maxit - 1, 0), &r2);
            } else {
                if (fell_back) *fell_back = 1;
                set_freestream(nullptr);
                shoot(tol, eta, maxit, &r2);
            }
        }
        if (rep) {
            pa_shoot_report r = converged ? r1 : r2;
            if (!converged) {
                r.newton_its += r1.newton_its;
                r.krylov_its += r1.krylov_its;
                r.primal_sweeps += r1.primal_sweeps;
                r.stage_newton_its += r1.stage_newton_its;
                r.stage_gmres_its += r1.stage_gmres_its;
                r.res0 = r1.res0;
                r.ms += r1.ms;
            }
            *rep = r;
        }
    }
    // the trained POD: mean deviation [Nu], modes [kmax][Nu], eigenvalues [kmax]
    int ws_pod(int kmax, double* mean, double* modes, double* eig) override
    {
        if (!ws_k) raise(PA_ESTATE, "no trained warm-start model");
        const int k = std::min(kmax, ws_k);
        if (mean) d2h(mean, ws_mean, sizeof(double) * Nu);
        if (modes && k > 0) d2h(modes, ws_psi, sizeof(double) * (size_t)k * Nu);
        if (eig)
            for (int j = 0; j < k; ++j) eig[j] = ws_lam[j];
        return ws_k;
    }
    void ws_save(const char* path) override
    {
        if (!ws_k) raise(PA_ESTATE, "no trained warm-start model");
        FILE* f = std::fopen(path, "wb");
        if (!f) raise(PA_EINVAL, "cannot write %s", path);
        std::vector<double> mean(Nu), psi((size_t)ws_k * Nu);
        std::vector<float> W(mlp.nparam);
        d2h(mean.data(), ws_mean, sizeof(double) * Nu);
        d2h(psi.data(), ws_psi, sizeof(double) * psi.size());
        d2h(W.data(), mlp.p, sizeof(float) * W.size());
        const char magic[8] = { 'P', 'A', 'W', 'S', '2', 0, 0, 0 };
        const int64_t hdr[3] = { Nu, ws_k, mlp.width() };
        bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(hdr, sizeof hdr, 1, f) == 1 &&
                  std::fwrite(ws_xm, sizeof ws_xm, 1, f) == 1 && std::fwrite(ws_xs, sizeof ws_xs, 1, f) == 1 &&
                  std::fwrite(ws_cs_h.data(), sizeof(float), ws_k, f) == (size_t)ws_k &&
                  std::fwrite(ws_lam.data(), sizeof(double), ws_k, f) == (size_t)ws_k &&
                  std::fwrite(mean.data(), sizeof(double), Nu, f) == (size_t)Nu &&
                  std::fwrite(psi.data(), sizeof(double), psi.size(), f) == psi.size() &&
                  std::fwrite(W.data(), sizeof(float), W.size(), f) == W.size();
        std::fclose(f);
        if (!ok) raise(PA_EINVAL, "short write to %s", path);
    }
    void ws_load(const char* path) override
    {
        FILE* f = std::fopen(path, "rb");
        if (!f) raise(PA_EINVAL, "cannot read %s", path);
        struct Close { FILE* f; ~Close() { std::fclose(f); } } cl{ f };
        char magic[8];
        int64_t hdr[3];
        if (std::fread(magic, 1, 8, f) != 8 || std::memcmp(magic, "PAWS2", 5) != 0) raise(PA_EINVAL, "not a warm-start file");
        if (std::fread(hdr, sizeof hdr, 1, f) != 1 || hdr[0] != Nu || hdr[1] < 1 || hdr[1] > WS_MAXK || hdr[2] < 1 ||
            hdr[2] > 4096)
            raise(PA_EINVAL, "warm-start file does not match this discretisation");
        const int k = (int)hdr[1], width = (int)hdr[2];
        std::vector<float> cs(k);
        std::vector<double> mean(Nu), psi((size_t)k * Nu), lam(k);
        float xm[WS_NIN], xs[WS_NIN];
        if (std::fread(xm, sizeof xm, 1, f) != 1 || std::fread(xs, sizeof xs, 1, f) != 1 ||
            std::fread(cs.data(), sizeof(float), k, f) != (size_t)k ||
            std::fread(lam.data(), sizeof(double), k, f) != (size_t)k ||
            std::fread(mean.data(), sizeof(double), Nu, f) != (size_t)Nu ||
            std::fread(psi.data(), sizeof(double), psi.size(), f) != psi.size())
            raise(PA_EINVAL, "truncated warm-start file");
        ws_alloc();
        mlp.init(WS_NIN, width, k, st);
        std::vector<float> W(mlp.nparam);
        if (std::fread(W.data(), sizeof(float), W.size(), f) != W.size()) raise(PA_EINVAL, "truncated warm-start file");
        h2d(mlp.p, W.data(), sizeof(float) * W.size());
        h2d(ws_mean, mean.data(), sizeof(double) * Nu);
        h2d(ws_psi, psi.data(), sizeof(double) * psi.size());
        h2d(ws_cs, cs.data(), sizeof(float) * k);
        ws_cs_h = cs;
        ws_lam = lam;
        std::memcpy(ws_xm, xm, sizeof xm);
        std::memcpy(ws_xs, xs, sizeof xs);
        ws_k = k;
    }

    // ---------------------------------------------------------------- several right-hand sides
    // R <= GM_RMAX systems with the same stage operator solved in lockstep:
    // one apply per iteration reads the stored blocks once for all R basis
    // vectors; the Arnoldi kernels run with one grid row per system; each
    // system has its own device GMRES state and stops on its own tolerance.
    int RM = 0;
    double *Vm = nullptr, *wm = nullptr, *ym = nullptr, *bm = nullptr, *rm = nullptr, *partm = nullptr;
    double *t1m = nullptr, *t2m = nullptr;                     // jprod temporaries
    double *lamm = nullptr, *rhsm = nullptr, *kapm = nullptr, *skm = nullptr, *fpm = nullptr, *drmm = nullptr;
    GmState* gmsm = nullptr;
    GmHost* hstm = nullptr;                                    // pinned [GM_RMAX]
    void ensure_multi()
    {
        if (RM) return;
        const int R = GM_RMAX;
        Vm = dalloc<double>((int64_t)R * (restart + 1) * Nu);
        wm = dalloc<double>(R * Nu); ym = dalloc<double>(R * Nu); bm = dalloc<double>(R * Nu);
        rm = dalloc<double>(R * Nu); t1m = dalloc<double>(R * Nu); t2m = dalloc<double>(R * Nu);
        lamm = dalloc<double>(R * Nu); rhsm = dalloc<double>(R * Nu); kapm = dalloc<double>(R * Nu);
        skm = dalloc<double>(3 * R * Nu); fpm = dalloc<double>(3 * R * Nu); drmm = dalloc<double>(3 * Nu);
        partm = dalloc<double>((int64_t)R * mdot_blocks(Nu) * (restart + 2));
        stgX = dalloc<double>(R * Nu); stgY = dalloc<double>(R * Nu); outm = dalloc<double>(R * Nu);
        brhs = dalloc<double>(R * Nu);
        gmsm = dalloc<GmState>(R);
        HIPCHK(hipHostMalloc((void**)&hstm, R * sizeof(GmHost), hipHostMallocDefault));
        RM = R;
    }
    // (Ahp: optional device slot holding the operator's address; such
    // launches, meant for graph capture, are not timed)
    void ahat_m(const double* Ah, int tr, int R, const double* x, int64_t sx, double* y, int64_t sy,
                const GmState* skip = nullptr, const double* const* Ahp = nullptr)
    {
        const int k = Ahp ? -1 : tr ? PA_K_SPMV_TM : PA_K_SPMV_M;
        switch (R) {
#define PA_AHAT_M(RR)                                                                                         \
    case RR:                                                                                                  \
        if (tr) klaunch(k, k_ahat_tr_m<NP, RR>, dim3(Ne), dim3(64), 0, Ne, nb4t, Ah, x, sx, y, sy, skip, Ahp); \
        else klaunch(k, k_ahat_fwd_m<NP, RR>, dim3(Ne), dim3(64), 0, Ne, nb4f, Ah, x, sx, y, sy, skip, Ahp);   \
        break;
            PA_AHAT_M(1) PA_AHAT_M(2) PA_AHAT_M(3) PA_AHAT_M(4) PA_AHAT_M(5) PA_AHAT_M(6) PA_AHAT_M(7) PA_AHAT_M(8)
#undef PA_AHAT_M
        default: raise(PA_EINVAL, "%d right-hand sides per apply (1..%d)", R, GM_RMAX);
        }
    }
    void poll_multi(int R)
    {
        for (int r = 0; r < R; ++r)
            HIPCHK(hipMemcpyAsync(&hstm[r], &gmsm[r].res, sizeof(GmHost), hipMemcpyDeviceToHost, st));
    }
    // x_r solves op(A) x_r = rhs_r, r < R; rhs and x hold R vectors at stride Nu
    int stage_solve_multi(const StageOps& op, int tr, int R, const double* rhs, double* x,
                          const double* x0 = nullptr)
    {
        if (R == 1 || pmode != PA_PREC_FP64) {
            int tot = 0;
            for (int r = 0; r < R; ++r) tot += stage_solve(op, tr, rhs + r * Nu, x + r * Nu, x0 ? x0 + r * Nu : nullptr);
            return tot;
        }
        if (R > GM_RMAX) raise(PA_EINVAL, "at most %d right-hand sides", GM_RMAX);
        ensure_multi();
        if (use_wg) return stage_solve_wg(op, tr, R, rhs, x, Vm, ym, wm);
        const int m = restart, maxit = 20 * restart;
        const int nb = (int)mdot_blocks(Nu);
        const int64_t sV = (int64_t)(m + 1) * Nu, sP = (int64_t)nb * (m + 2);
        const double* b = rhs;
        if (tr) {
            for (int r = 0; r < R; ++r) prec(op.Pinv, 1, rhs + r * Nu, bm + r * Nu);
            b = bm;
        }
        double bn[GM_RMAX], tol[GM_RMAX];
        bool acc[GM_RMAX];
        GmTol tl{};
        for (int r = 0; r < R; ++r) {
            bn[r] = norm(b + r * Nu);
            tol[r] = cfg.lin_rtol * bn[r];
            acc[r] = bn[r] == 0.0;
            tl.t[r] = acc[r] ? 1e300 : tol[r];
        }
        if (x0) {   // per system: the guess when its residual is below |b_r|, else zero
            for (int r = 0; r < R; ++r) {
                if (tr) copy(x0 + r * Nu, ym + r * Nu);
                else prec(op.Pd, 0, x0 + r * Nu, ym + r * Nu);
            }
            ahat_m(op.Ah, tr, R, ym, Nu, wm, Nu);
            for (int r = 0; r < R; ++r) {
                lincomb(1.0, b + r * Nu, -1.0, wm + r * Nu, rm + r * Nu);
                ++cnt_guess_try;
                if (norm(rm + r * Nu) < bn[r]) {
                    ++cnt_guess_used;
                } else {
                    zero(ym + r * Nu);
                    copy(b + r * Nu, rm + r * Nu);
                }
            }
        } else {
            zero(ym, R * Nu);
            HIPCHK(hipMemcpyAsync(rm, b, sizeof(double) * R * Nu, hipMemcpyDeviceToDevice, st));
        }
        int total = 0;
        bool all = true;
        for (int r = 0; r < R; ++r) all = all && acc[r];
        if (use_graph && !all) set_graph_op(op.Ah);
        while (!all) {
            const dim3 g2(nb, R);
            k_mdot_part<<<g2, MD_THREADS, 0, st>>>(rm, 0, 1, 0, rm, Nu, partm, nullptr, Nu, Nu, sP);
            k_gm_begin<<<g2, MD_THREADS, 0, st>>>(rm, Vm, Nu, partm, nb, tl, gmsm, Nu, sV, sP);
            LAUNCHCHK();
            int pending = -1, jlast = 0;
            hipEvent_t ev_p = nullptr;
            for (int j = 0; j < m; ++j) {
                jlast = j;
                if (use_graph) {
                    // iterations j .. j + GM_CHECK - 1 (m is a multiple of GM_CHECK)
                    if (j % GM_CHECK == 0) HIPCHK(hipGraphLaunch(gm_graph(tr, R, j / GM_CHECK), st));
                } else {
                    ahat_m(op.Ah, tr, R, Vm + (int64_t)j * Nu, sV, wm, Nu, gmsm);
                    klaunch(PA_K_MDOT, k_mdot_part<double>, dim3(nb, mdot_chunks(j + 2) * R), dim3(MD_THREADS), 0, Vm,
                            Nu, j + 1, 1, wm, Nu, partm, gmsm, sV, Nu, sP);
                    klaunch(PA_K_GMUPD, k_gm_upd<double>, dim3((unsigned)gm_upd_blocks(Nu), R), dim3(GU_THREADS), 0, Vm,
                            Nu, j, m, wm, Nu, partm, nb, gmsm, sV, Nu, sP);
                }
                if ((j + 1) % GM_CHECK == 0 && j < m - 1) {
                    if (pending >= 0) {
                        HIPCHK(hipEventSynchronize(ev_p));
                        bool alldone = true;
                        for (int r = 0; r < R; ++r) alldone = alldone && hstm[r].done;
                        if (alldone) break;
                    }
                    poll_multi(R);
                    HIPCHK(hipEventRecord(gm_ev[0], st));
                    ev_p = gm_ev[0];
                    pending = 0;
                }
            }
            k_gm_solve<<<R, 256, 0, st>>>(m, gmsm);
            k_gm_combine<<<dim3(grid1(Nu), R), 256, 0, st>>>(Vm, Nu, m, wm, Nu, gmsm, sV, Nu);
            LAUNCHCHK();
            poll_multi(R);
            for (int r = 0; r < R; ++r)
                if (!acc[r]) axpby(1.0, wm + r * Nu, 1.0, ym + r * Nu);
            ahat_m(op.Ah, tr, R, ym, Nu, wm, Nu);
            for (int r = 0; r < R; ++r) lincomb(1.0, b + r * Nu, -1.0, wm + r * Nu, rm + r * Nu);
            all = true;
            int cyc = 0;
            for (int r = 0; r < R; ++r) {
                const double rn = norm(rm + r * Nu);   // synchronises: hstm valid
                if (!acc[r]) {
                    cyc = std::max(cyc, hstm[r].done ? hstm[r].its : m);
                    tvec_cycle(hstm[r].done ? hstm[r].its : m);
                    if (!std::isfinite(rn) || !std::isfinite(hstm[r].res)) raise(PA_ENUMERIC, "NaN in stage GMRES");
                    if (hstm[r].done && rn <= 2.0 * tol[r]) { acc[r] = true; tl.t[r] = 1e300; }
                }
                all = all && acc[r];
            }
            total += cyc;
            // the applies and vector kernels of the cycle return at once when
            // every system is done
            tskip(tr ? PA_K_SPMV_TM : PA_K_SPMV_M, jlast + 1 - cyc);
            tskip(PA_K_MDOT, jlast + 1 - cyc);
            tskip(PA_K_GMUPD, jlast + 1 - cyc);
            if (!all && total >= maxit) raise(PA_ENOCONV, "stage GMRES (%d systems) did not converge in %d iterations", R, total);
        }
        for (int r = 0; r < R; ++r) {
            if (tr) copy(ym + r * Nu, x + r * Nu);
            else prec(op.Pinv, 0, ym + r * Nu, x + r * Nu);
        }
        cnt_gmres += (int64_t)total * R;
        return total;
    }
    // out_r = dt J^T w_r (transposed stage Jacobian products, R systems)
    void stage_jprod_tr_multi(const StageOps& op, int R, const double* w, double* out)
    {
        ahat_m(op.Ah, 1, R, w, Nu, t1m, Nu);
        const double ia = dt / op.aii;
        for (int r = 0; r < R; ++r) {
            prec(op.Pd, 1, t1m + r * Nu, t2m + r * Nu);
            k_mass_axpy<NP><<<grid1(Nu), 256, 0, st>>>(Ne, dm.area, dmh, w + r * Nu, t2m + r * Nu, ia, -ia, out + r * Nu);
        }
        LAUNCHCHK();
    }
    // forward stage Jacobian products out_r = dt J w_r for R systems
    void stage_jprod_fwd_multi(const StageOps& op, int R, const double* w, double* out)
    {
        for (int r = 0; r < R; ++r) prec(op.Pd, 0, w + r * Nu, t1m + r * Nu);
        ahat_m(op.Ah, 0, R, t1m, Nu, t2m, Nu);
        const double ia = dt / op.aii;
        for (int r = 0; r < R; ++r)
            k_mass_axpy<NP><<<grid1(Nu), 256, 0, st>>>(Ne, dm.area, dmh, w + r * Nu, t2m + r * Nu, ia, -ia, out + r * Nu);
        LAUNCHCHK();
    }
    // tangent sweeps of R systems together: out_r = Phi v_r, plus (mu_dir[r]
    // >= 0) the forcing dt dr/dmu_k of a parameter tangent (Sec. 2.2 eq.
    // dirk-sens-mvp with the parameter term), and (dq != NULL) the tangent of
    // both time-averaged QoIs: dq[2 r + q] = sum_n sum_i dt b_i / T
    // (df_q/du(u_i) du_i + df_q/dmu_k), du_i = w_i + a_ii dk_i
    void tangent_multi(int R, const double* v, const int* mu_dir, double* out, double* dq)
    {
        if (!have_traj) raise(PA_ESTATE, "no trajectory");
        if (R > GM_RMAX) raise(PA_EINVAL, "at most %d right-hand sides", GM_RMAX);
        ensure_multi();
        double* du = lamm;
        double* w = rhsm;
        double* rhs = kapm;
        auto DK = [&](int i, int r) { return skm + ((int64_t)i * R + r) * Nu; };
        HIPCHK(hipMemcpyAsync(du, v, sizeof(double) * R * Nu, hipMemcpyDeviceToDevice, st));
        bool forced = false;
        for (int r = 0; r < R; ++r) forced = forced || mu_dir[r] >= 0;
        std::vector<double> acc(2 * R, 0.0);
        double* qg = fpm;            // df_q/du, q = 0, 1 (two vectors)
        double* dui = fpm + 2 * Nu;  // du_i of one system
        const double sc = dt / cfg.T;
        for (int n = 1; n <= Nt; ++n) {
            for (int i = 1; i <= 3; ++i) {
                const int s = (n - 1) * 3 + (i - 1);
                for (int r = 0; r < R; ++r) {
                    copy(du + r * Nu, w + r * Nu);
                    for (int j = 1; j < i; ++j) axpby(rk.A[i - 1][j - 1], DK(j - 1, r), 1.0, w + r * Nu);
                }
                stage_jprod_fwd_multi(ops(s), R, w, rhs);
                if (forced) {
                    dr_dmu(n, i, stU(s), drmm);
                    for (int r = 0; r < R; ++r)
                        if (mu_dir[r] >= 0) axpby(dt, drmm + (int64_t)mu_dir[r] * Nu, 1.0, rhs + r * Nu);
                }
                stage_solve_multi(ops(s), 0, R, rhs, DK(i - 1, 0), cfg.lin_guess && n > 1 ? DK(i - 1, 0) : nullptr);
                if (dq) {
                    qoi_grad(n, i, stU(s), 0, qg, qtmp);
                    qoi_grad(n, i, stU(s), 1, qg + Nu, qtmp);
                    double fm[6] = { 0, 0, 0, 0, 0, 0 };
                    if (forced) qoi_dmu(n, i, stU(s), fm, nullptr);
                    for (int r = 0; r < R; ++r) {
                        lincomb(1.0, w + r * Nu, rk.A[i - 1][i - 1], DK(i - 1, r), dui);
                        double d[2];
                        dots(qg, Nu, 2, dui, d);
                        for (int q = 0; q < 2; ++q) {
                            double t = d[q];
                            if (mu_dir[r] >= 0) t += fm[3 * q + mu_dir[r]];
                            acc[2 * r + q] += sc * rk.b[i - 1] * t;
                        }
                    }
                }
            }
            for (int r = 0; r < R; ++r)
                for (int i = 0; i < 3; ++i) axpby(rk.b[i], DK(i, r), 1.0, du + r * Nu);
        }
        HIPCHK(hipMemcpyAsync(out, du, sizeof(double) * R * Nu, hipMemcpyDeviceToDevice, st));
        if (dq) for (int k = 0; k < 2 * R; ++k) dq[k] = acc[k];
    }

    // backward sweeps of R systems together (as adjoint()): lamNt, lam0 hold R
    // vectors; system r is forced by QoI fq[r] >= 0 (then grad[3 r + k])
    void adjoint_multi(int R, const double* lamNt, const int* fq, double* lam0, double* grad)
    {
        if (!have_traj) raise(PA_ESTATE, "no trajectory");
        if (R == 1) { adjoint(lamNt, fq[0], lam0, grad); return; }
        ensure_multi();
        if (R > GM_RMAX) raise(PA_EINVAL, "at most %d right-hand sides", GM_RMAX);
        double* lam = lamm;
        double* rhs = rhsm;
        if (!kap3m) kap3m = dalloc<double>((int64_t)3 * GM_RMAX * Nu);
        auto SK = [&](int i, int r) { return skm + ((int64_t)i * R + r) * Nu; };
        auto FP = [&](int i, int r) { return fpm + ((int64_t)i * R + r) * Nu; };
        HIPCHK(hipMemcpyAsync(lam, lamNt, sizeof(double) * R * Nu, hipMemcpyDeviceToDevice, st));
        std::vector<double> g(3 * R, 0.0);
        bool anyf = false;
        for (int r = 0; r < R; ++r) anyf = anyf || fq[r] >= 0;
        const double sc = dt / cfg.T;
        for (int n = Nt; n >= 1; --n) {
            for (int r = 0; r < R; ++r) {
                if (fq[r] < 0) continue;
                for (int i = 1; i <= 3; ++i) {
                    const int s = (n - 1) * 3 + (i - 1);
                    qoi_grad(n, i, stU(s), fq[r], FP(i - 1, r), qtmp);
                    double fm[6];
                    qoi_dmu(n, i, stU(s), fm, nullptr);
                    for (int k = 0; k < 3; ++k) g[3 * r + k] += sc * rk.b[i - 1] * fm[3 * fq[r] + k];
                }
            }
            for (int i = 3; i >= 1; --i) {
                const int s = (n - 1) * 3 + (i - 1);
                for (int r = 0; r < R; ++r) {
                    double* rr = rhs + r * Nu;
                    lincomb(rk.b[i - 1], lam + r * Nu, 0.0, lam + r * Nu, rr);
                    for (int j = i + 1; j <= 3; ++j) axpby(rk.A[j - 1][i - 1], SK(j - 1, r), 1.0, rr);
                    if (fq[r] >= 0)
                        for (int j = i; j <= 3; ++j) axpby(sc * rk.b[j - 1] * rk.A[j - 1][i - 1], FP(j - 1, r), 1.0, rr);
                }
                double* kap = kap3m + (int64_t)(i - 1) * R * Nu;   // this stage's multipliers (the guess)
                stage_solve_multi(ops(s), 1, R, rhs, kap, cfg.lin_guess && n < Nt ? kap : nullptr);
                // dt J^T kap_r into the stage slots (contiguous per stage)
                stage_jprod_tr_multi(ops(s), R, kap, SK(i - 1, 0));
                if (anyf) {
                    dr_dmu(n, i, stU(s), drmm);
                    for (int r = 0; r < R; ++r) {
                        if (fq[r] < 0) continue;
                        double d[3];
                        dots(drmm, Nu, 3, kap + r * Nu, d);
                        for (int k = 0; k < 3; ++k) g[3 * r + k] += dt * d[k];
                    }
                }
            }
            for (int r = 0; r < R; ++r) {
                for (int i = 0; i < 3; ++i) axpby(1.0, SK(i, r), 1.0, lam + r * Nu);
                if (fq[r] >= 0)
                    for (int i = 0; i < 3; ++i) axpby(sc * rk.b[i], FP(i, r), 1.0, lam + r * Nu);
            }
        }
        HIPCHK(hipMemcpyAsync(lam0, lam, sizeof(double) * R * Nu, hipMemcpyDeviceToDevice, st));
        if (grad) for (int k = 0; k < 3 * R; ++k) grad[k] = g[k];
    }

    // out = dt J op(w) of a stage:  c J = M - A,  A = Ahat P,  A^T = P^T Ahat^T
    void stage_jprod(const StageOps& op, int tr, const double* w, double* out, double* tmp1, double* tmp2)
    {
        if (!tr) {
            prec(op.Pd, 0, w, tmp1);
            ahat(op.Ah, 0, tmp1, tmp2);
        } else {
            ahat(op.Ah, 1, w, tmp1);
            prec(op.Pd, 1, tmp1, tmp2);
        }
        // dt J w = (dt / c)(M w - A w) = (M w - A w) / a_ii
        const double ia = dt / op.aii;
        k_mass_axpy<NP><<<grid1(Nu), 256, 0, st>>>(Ne, dm.area, dmh, w, tmp2, ia, -ia, out);
        LAUNCHCHK();
    }
    GmState* gms = nullptr;
    GmHost* hstat = nullptr;       // pinned: two check slots and the end-of-cycle status
    bool use_wg = false;           // FP64 stage solves in one workgroup per system (small meshes)
    double* kap3 = nullptr;        // adjoint sweep: the multipliers of the three stages of a step
    double* kap3m = nullptr;       // the same for several systems [3][GM_RMAX][Nu]
    WgStatus* wgst = nullptr;      // device [GM_RMAX]
    WgStatus* hwgst = nullptr;     // pinned copy
    hipEvent_t gm_ev[2] = {nullptr, nullptr};

    // ---------------------------------------------------------------- setup
    void set_params(const double m[3]) override
    {
        std::memcpy(mu, m, sizeof mu);
        have_params = true;
        have_traj = false;
        // gbar(0) and its mu-derivatives
        k_gbar0<P, Dual<3>><<<Ne, 64, 0, st>>>(dm, dref, motion_d(0.0), rg4, nn);
        LAUNCHCHK();
        HIPCHK(hipMemcpyAsync(gb, rg4, sizeof(double) * nn, hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemcpyAsync(dgb, rg4 + nn, sizeof(double) * 3 * nn, hipMemcpyDeviceToDevice, st));
        for (int n = 1; n <= Nt; ++n) {
            const int prev = gidx(n - 1, n - 1 == 0 ? 0 : 3);
            for (int i = 1; i <= 3; ++i) {
                k_gcl_rhs<P, Dual<3>><<<Ne, 64, 0, st>>>(dm, dref, motion_d(stage_time(n, i)), rg4, nn);
                LAUNCHCHK();
                k_gcl_kstage<P><<<grid1(4 * nn), 256, 0, st>>>(dm, dref, rg4, dt, kg4 + (int64_t)(i - 1) * 4 * nn, 4, nn);
                LAUNCHCHK();
                const int cur = gidx(n, i);
                // value field and the three derivative fields
                for (int fld = 0; fld < 4; ++fld) {
                    double* dst = fld == 0 ? gb + (int64_t)cur * nn : dgb + ((int64_t)cur * 3 + fld - 1) * nn;
                    const double* src = fld == 0 ? gb + (int64_t)prev * nn : dgb + ((int64_t)prev * 3 + fld - 1) * nn;
                    HIPCHK(hipMemcpyAsync(dst, src, sizeof(double) * nn, hipMemcpyDeviceToDevice, st));
                    for (int j = 1; j <= i; ++j) {
                        k_axpby<<<grid1(nn), 256, 0, st>>>(rk.A[i - 1][j - 1], kg4 + ((int64_t)(j - 1) * 4 + fld) * nn,
                                                            1.0, dst, nn);
                        LAUNCHCHK();
                    }
                }
            }
        }
        HIPCHK(hipStreamSynchronize(st));
    }

    void set_state(const double* h, int64_t n) override
    {
        if (n != Nu) raise(PA_EINVAL, "state length %lld != %lld", (long long)n, (long long)Nu);
        h2d(u0, h, sizeof(double) * Nu);
        have_traj = false;
    }
    void set_freestream(const double* pert) override
    {
        if (!have_params) raise(PA_ESTATE, "parameters not set");
        std::vector<double> g(nn), u(Nu);
        d2h(g.data(), gb, sizeof(double) * nn);
        for (int64_t k = 0; k < nn; ++k)
            for (int m = 0; m < 4; ++m) u[4 * k + m] = g[k] * ph.Uinf[m] + (pert ? pert[4 * k + m] : 0.0);
        set_state(u.data(), Nu);
    }
    void get_state(int which, double* out, int64_t n) override
    {
        if (n != Nu) raise(PA_EINVAL, "bad length");
        if (which == 0) d2h(out, u0, sizeof(double) * Nu);
        else if (which == 1) {
            if (!have_traj) raise(PA_ESTATE, "no trajectory");
            d2h(out, tu + (int64_t)Nt * Nu, sizeof(double) * Nu);
        } else raise(PA_EINVAL, "bad which");
    }

    // ---------------------------------------------------------------- sweeps
    // stage QoI values of all wall elements into qh[s]
    void qoi_values(int n, int i, const double* u, double* fval)
    {
        if (!nwall) return;
        k_qoi_du<P><<<grid1((int64_t)nwall * B, 64), 64, 0, st>>>(dm, dref, ph, motion(stage_time(n, i)), dwall, nwall,
                                                                  u, gbs(n, i), fval, qdu);
        LAUNCHCHK();
    }
    // dense df_q/du [Nu] of QoI q at stage (n, i) into out
    void qoi_grad(int n, int i, const double* u, int q, double* out, double* fval)
    {
        zero(out);
        if (!nwall) return;
        k_qoi_du<P><<<grid1((int64_t)nwall * B, 64), 64, 0, st>>>(dm, dref, ph, motion(stage_time(n, i)), dwall, nwall,
                                                                  u, gbs(n, i), fval, qdu);
        LAUNCHCHK();
        for (int w = 0; w < nwall; ++w)
            HIPCHK(hipMemcpyAsync(out + (int64_t)wall[w] * B, qdu + ((int64_t)w * 2 + q) * B, sizeof(double) * B,
                                  hipMemcpyDeviceToDevice, st));
    }
    // explicit mu-derivative of the QoIs at a stage, host out[2][3] (and values)
    void qoi_dmu(int n, int i, const double* u, double out[6], double val[2])
    {
        for (int k = 0; k < 6; ++k) out[k] = 0.0;
        if (val) val[0] = val[1] = 0.0;
        if (!nwall) return;
        k_qoi_dmu<P><<<grid1(nwall, 64), 64, 0, st>>>(dm, dref, ph, motion_d(stage_time(n, i)), dwall, nwall, u, gbs(n, i),
                                                      dgbs(n, i), qdmu, nn);
        LAUNCHCHK();
        std::vector<double> h((size_t)nwall * 8);
        HIPCHK(hipMemcpyAsync(h.data(), qdmu, sizeof(double) * h.size(), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        for (int w = 0; w < nwall; ++w)
            for (int q = 0; q < 2; ++q) {
                if (val) val[q] += h[8 * w + 4 * q];
                for (int k = 0; k < 3; ++k) out[3 * q + k] += h[8 * w + 4 * q + 1 + k];
            }
    }

    StageOps ops(int s) const
    {
        const void* al = nullptr;
        if (pmode == PA_PREC_FP32) al = (const float*)tAl + (int64_t)s * 3 * Isz;
        else if (pmode == PA_PREC_BF16) al = (const bf16_t*)tAl + (int64_t)s * 3 * Isz;
        return { tAh + (int64_t)s * 3 * Isz, tPd + (int64_t)s * Isz, tAi + (int64_t)s * Isz,
                 dt * rk.A[s % 3][s % 3], al };
    }
    // dr/du at (n, i, u) -> Jtmp, then P, P^{-1} and Ahat of A = M - c J into stage slot s
    void assemble(int n, int i, const double* u, double c, int s)
    {
        jacobian(n, i, u, Jtmp);
        prepare_ops(Jtmp, c, s);
    }
    void prepare_ops(const double* J, double c, int s)
    {
        // timed from the start of the first kernel to the end of the second
        hipEvent_t ea, eb;
        tsample(PA_K_BLOCKINV, &ea, &eb);
        klaunch_ev(ea, nullptr, k_blockprep<NP>, dim3(Ne), dim3(64), 0, Ne, dm.area, dmh, J, c, tPd + (int64_t)s * Isz,
                   tAi + (int64_t)s * Isz, dstatus);
        klaunch_ev(nullptr, eb, k_form_ahat_mfma<NP>, dim3(Ne * 3), dim3(64), 0, Ne, dm.enb, J, c,
                   tAi + (int64_t)s * Isz, tAh + (int64_t)s * 3 * Isz);
        if (cfg.autotune && !fwd_tuned) tune_fwd(tAh + (int64_t)s * 3 * Isz);
        const int64_t n3 = 3 * Isz;
        if (pmode == PA_PREC_FP32)
            k_to_lo<float><<<grid1(n3), 256, 0, st>>>(tAh + s * n3, (float*)tAl + s * n3, n3);
        else if (pmode == PA_PREC_BF16)
            k_to_lo<bf16_t><<<grid1(n3), 256, 0, st>>>(tAh + s * n3, (bf16_t*)tAl + s * n3, n3);
        LAUNCHCHK();
    }
    double* stK(int s) { return tk + (int64_t)s * Nu; }
    double* stU(int s) { return tui + (int64_t)s * Nu; }

    // primal period from u0 (device), Newton per stage
    void primal_sweep(double qoi[2], double* res)
    {
        if (!have_params) raise(PA_ESTATE, "parameters not set");
        have_traj = false;
        copy(u0, tu);
        done_stages = 0;
        double* ubase = wa;
        double* R = wb;
        double* dk = wc;
        double* r = wd;
        for (int n = 1; n <= Nt; ++n) {
            const double* uprev = tu + (int64_t)(n - 1) * Nu;
            for (int i = 1; i <= 3; ++i) {
                const int s = (n - 1) * 3 + (i - 1);
                const double aii = rk.A[i - 1][i - 1], c = dt * aii;
                copy(uprev, ubase);
                for (int j = 1; j < i; ++j) axpby(rk.A[i - 1][j - 1], stK(s - i + j), 1.0, ubase);
                double* k = stK(s);
                double* ui = stU(s);
                double* kt = we;   // trial slope; the stage GMRES is idle while it is live
                auto evalR = [&](const double* kk) {
                    lincomb(1.0, ubase, aii, kk, ui);
                    residual(n, i, ui, r);
                    k_stage_residual<NP><<<grid1(Nu), 256, 0, st>>>(Ne, dm.area, dmh, kk, r, dt, R);
                    LAUNCHCHK();
                    return norm(R);
                };
                // predictor: previous stage slope, or the slope that places u_i
                // at the previous stage state -- whichever has the smaller
                // Newton residual (the slope on ties); zero at the first stage
                double nR;
                if (s > 0) {
                    lincomb(1.0 / aii, stU(s - 1), -1.0 / aii, ubase, kt);
                    double n2 = evalR(kt);
                    copy(stK(s - 1), k);
                    nR = evalR(k);
                    if (!(nR <= n2)) { copy(kt, k); nR = evalR(k); }
                } else {
                    zero(k);
                    nR = evalR(k);
                }
                if (verbose > 1) fprintf(stderr, "[pa] stage (%d,%d) predictor |R| = %.3e\n", n, i, nR);
                int it = 0;
                while (!(nR <= cfg.newton_atol)) {
                    if (!std::isfinite(nR)) raise(PA_ENUMERIC, "NaN at stage (%d,%d)", n, i);
                    if (it >= cfg.newton_maxit)
                        raise(PA_ENOCONV, "stage Newton did not converge at (%d,%d): |R| = %.3e", n, i, nR);
                    assemble(n, i, ui, c, s);
                    stage_solve(ops(s), 0, R, dk);
                    // backtracking on ||R||: halve until it decreases (NaN counts as no decrease)
                    double lam = 1.0, nT;
                    for (;;) {
                        lincomb(1.0, k, -lam, dk, kt);
                        nT = evalR(kt);
                        if (nT < nR) break;
                        lam *= 0.5;
                        if (lam < 1e-4) raise(PA_ENOCONV, "line search failed at stage (%d,%d), |R| = %.3e", n, i, nR);
                    }
                    copy(kt, k);
                    nR = nT;
                    ++it;
                    ++cnt_newton;
                    if (verbose > 1) fprintf(stderr, "[pa] stage (%d,%d) it %d lam %.3g |R| = %.3e\n", n, i, it, lam, nR);
                }
                // exact linearisation at the converged stage state
                assemble(n, i, ui, c, s);
                qoi_values(n, i, ui, qh + (int64_t)s * std::max(nwall, 1) * 2);
                done_stages = s + 1 - (i == 3 ? 1 : 0);   // u^(n) is written after the step
            }
            double* un = tu + (int64_t)n * Nu;
            copy(uprev, un);
            for (int i = 0; i < 3; ++i) axpby(rk.b[i], stK((n - 1) * 3 + i), 1.0, un);
            done_stages = 3 * n;
        }
        // time-averaged QoIs (fixed-order host sum)
        std::vector<double> h((size_t)nst * std::max(nwall, 1) * 2);
        HIPCHK(hipMemcpyAsync(h.data(), qh, sizeof(double) * h.size(), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        double J0 = 0, J1 = 0;
        for (int s = 0; s < nst; ++s) {
            double f0 = 0, f1 = 0;
            for (int w = 0; w < nwall; ++w) { f0 += h[((size_t)s * nwall + w) * 2]; f1 += h[((size_t)s * nwall + w) * 2 + 1]; }
            J0 += dt * rk.b[s % 3] * f0 / cfg.T;
            J1 += dt * rk.b[s % 3] * f1 / cfg.T;
        }
        if (qoi) { qoi[0] = J0; qoi[1] = J1; }
        last_qoi[0] = J0;
        last_qoi[1] = J1;
        lincomb(1.0, tu + (int64_t)Nt * Nu, -1.0, u0, wa);
        double rn = norm(wa);
        if (res) *res = rn;
        have_traj = true;
    }

    void primal_period(double qoi[2], double* res) override { primal_sweep(qoi, res); }
    double last_qoi[2] = { 0, 0 };   // time-averaged QoIs of the last primal sweep
    void last_qois(double q[2]) const override { q[0] = last_qoi[0]; q[1] = last_qoi[1]; }

    // tangent sweep: out = Phi v (device vectors; out may alias nothing used here)
    void tangent(const double* v, double* out)
    {
        if (!have_traj) raise(PA_ESTATE, "no trajectory");
        double* du = wa;
        double* w = wb;
        double* rhs = wc;
        copy(v, du);
        for (int n = 1; n <= Nt; ++n) {
            for (int i = 1; i <= 3; ++i) {
                const int s = (n - 1) * 3 + (i - 1);
                copy(du, w);
                for (int j = 1; j < i; ++j) axpby(rk.A[i - 1][j - 1], sk3 + (int64_t)(j - 1) * Nu, 1.0, w);
                stage_jprod(ops(s), 0, w, rhs, gm_b, gm_y);
                // guess: the same stage's slope one step earlier (still in sk3)
                double* ki = sk3 + (int64_t)(i - 1) * Nu;
                stage_solve(ops(s), 0, rhs, ki, cfg.lin_guess && n > 1 ? ki : nullptr);
            }
            for (int i = 0; i < 3; ++i) axpby(rk.b[i], sk3 + (int64_t)i * Nu, 1.0, du);
        }
        copy(du, out);
    }

    // backward adjoint sweep from lamNt; forced by QoI fq >= 0 (then grad[3])
    void adjoint(const double* lamNt, int fq, double* lam0, double* grad)
    {
        if (!have_traj) raise(PA_ESTATE, "no trajectory");
        double* lam = wa;
        double* rhs = wb;
        if (!kap3) kap3 = dalloc<double>(3 * Nu);
        copy(lamNt, lam);
        double g[3] = { 0, 0, 0 };
        const double sc = dt / cfg.T;
        for (int n = Nt; n >= 1; --n) {
            if (fq >= 0)
                for (int i = 1; i <= 3; ++i) {
                    const int s = (n - 1) * 3 + (i - 1);
                    qoi_grad(n, i, stU(s), fq, fp3 + (int64_t)(i - 1) * Nu, qtmp);
                    double fm[6];
                    qoi_dmu(n, i, stU(s), fm, nullptr);
                    for (int k = 0; k < 3; ++k) g[k] += sc * rk.b[i - 1] * fm[3 * fq + k];
                }
            for (int i = 3; i >= 1; --i) {
                const int s = (n - 1) * 3 + (i - 1);
                lincomb(rk.b[i - 1], lam, 0.0, lam, rhs);
                for (int j = i + 1; j <= 3; ++j) axpby(rk.A[j - 1][i - 1], sk3 + (int64_t)(j - 1) * Nu, 1.0, rhs);
                if (fq >= 0)
                    for (int j = i; j <= 3; ++j)
                        axpby(sc * rk.b[j - 1] * rk.A[j - 1][i - 1], fp3 + (int64_t)(j - 1) * Nu, 1.0, rhs);
                // guess: the same stage's multiplier one step later
                double* kap = kap3 + (int64_t)(i - 1) * Nu;
                stage_solve(ops(s), 1, rhs, kap, cfg.lin_guess && n < Nt ? kap : nullptr);
                stage_jprod(ops(s), 1, kap, sk3 + (int64_t)(i - 1) * Nu, gm_b, gm_y);
                if (fq >= 0) {
                    dr_dmu(n, i, stU(s), drm);
                    double d[3];
                    dots(drm, Nu, 3, kap, d);
                    for (int k = 0; k < 3; ++k) g[k] += dt * d[k];
                }
            }
            for (int i = 0; i < 3; ++i) axpby(1.0, sk3 + (int64_t)i * Nu, 1.0, lam);
            if (fq >= 0)
                for (int i = 0; i < 3; ++i) axpby(sc * rk.b[i], fp3 + (int64_t)i * Nu, 1.0, lam);
        }
        copy(lam, lam0);
        if (grad) for (int k = 0; k < 3; ++k) grad[k] = g[k];
    }

    // ---------------------------------------------------------------- outer solvers
    // Newton-Krylov shooting with a backtracking line search on ||R||: the
    // step u0 - lam Delta is accepted when its primal period succeeds and
    // lowers the periodicity residual (lam = 1, 1/2, ... 1/64)
    void shoot(double tol, double eta, int maxit, pa_shoot_report* rep) override
    {
        double t0 = now_ms();
        pa_shoot_report r{};
        if (rep) {   // the caller's history buffers
            r.res_hist = rep->res_hist;
            r.krylov_hist = rep->krylov_hist;
            r.step_hist = rep->step_hist;
            r.hist_cap = rep->hist_cap;
        }
        cnt_newton = cnt_gmres = 0;
        auto finish = [&]() {
            r.stage_newton_its = (int32_t)cnt_newton;
            r.stage_gmres_its = cnt_gmres;
            r.ms = now_ms() - t0;
            if (rep) *rep = r;
        };
        double qoi[2], res;
        primal_sweep(qoi, &res);
        ++r.primal_sweeps;
        r.res0 = r.res = res;
        if (r.res_hist && r.hist_cap > 0) r.res_hist[0] = res;
        if (verbose) fprintf(stderr, "[pa] shoot start |R| = %.3e  %.1f s\n", res, (now_ms() - t0) / 1e3);
        while (!(res <= tol)) {
            if (r.newton_its >= maxit) {
                finish();
                raise(PA_ENOCONV, "shooting did not converge: |R| = %.3e after %d Newton steps", res, r.newton_its);
            }
            // R = u^(Nt) - u0;  (Phi - I) Delta = R
            lincomb(1.0, tu + (int64_t)Nt * Nu, -1.0, u0, wd);
            int k0 = r.krylov_its;
            outer_gmres(true, wd, eta, r.krylov_its);
            copy(wf, nk_delta);
            copy(u0, nk_save);
            double lam = 1.0, rnew = 0.0;
            bool ok = false;
            for (int trial = 0; trial < 7 && !ok; ++trial, lam *= 0.5) {
                lincomb(1.0, nk_save, -lam, nk_delta, u0);
                try {
                    primal_sweep(qoi, &rnew);
                    ++r.primal_sweeps;
                    ok = rnew < res;
                } catch (const PaError& e) {
                    if (e.code != PA_ENOCONV && e.code != PA_ENUMERIC) throw;
                    ++r.primal_sweeps;
                    ok = false;
                }
                if (verbose)
                    fprintf(stderr, "[pa] shoot it %d lam %.4g |R| = %.3e -> %s  %.1f s\n", r.newton_its + 1, lam,
                            res, ok ? "accepted" : "rejected", (now_ms() - t0) / 1e3);
                if (ok) break;
            }
            if (!ok) {
                copy(nk_save, u0);
                primal_sweep(qoi, &res);
                ++r.primal_sweeps;
                finish();
                raise(PA_ENOCONV, "shooting line search failed at |R| = %.3e", res);
            }
            res = rnew;
            r.res = res;
            const int k = r.newton_its;
            if (k < r.hist_cap) {
                if (r.krylov_hist) r.krylov_hist[k] = r.krylov_its - k0;
                if (r.step_hist) r.step_hist[k] = lam;
            }
            if (k + 1 < r.hist_cap && r.res_hist) r.res_hist[k + 1] = res;
            ++r.newton_its;
            if (verbose)
                fprintf(stderr, "[pa] shoot it %d |R| = %.3e (krylov %d, rel %.2e)  %.1f s\n", r.newton_its, res,
                        r.krylov_its - k0, last_outer_rel, (now_ms() - t0) / 1e3);
        }
        finish();
    }

    // Floquet multipliers of the stored trajectory (Sec. 2.3 discusses the
    // spectrum of Phi): k steps of Arnoldi on Phi with tangent sweeps from a
    // seeded random start (two Gram-Schmidt passes), then the eigenvalues of
    // the k x k Hessenberg matrix (Ritz values), sorted by modulus, largest
    // first.  Returns the basis size reached (smaller on an invariant
    // subspace); *hsub receives the last subdiagonal entry h_{k+1,k}.
    int floquet(int k, uint64_t seed, double* re, double* im, double* hsub) override
    {
        if (!have_traj) raise(PA_ESTATE, "no trajectory (run pa_primal_period or pa_shoot first)");
        if (k < 1 || k > max_kry) raise(PA_EINVAL, "basis size must be 1..max_krylov (%d)", max_kry);
        const int m = k;
        std::vector<double> H((size_t)(m + 1) * m, 0.0), h(m + 2), h2(m + 2);
        std::vector<double> v0(Nu);
        for (int64_t i = 0; i < Nu; ++i) v0[i] = (double)(splitmix64(seed) >> 11) * (1.0 / 9007199254740992.0) - 0.5;
        h2d(outer_w, v0.data(), sizeof(double) * Nu);
        const double n0 = norm(outer_w);
        lincomb(1.0 / n0, outer_w, 0.0, outer_w, Vo);
        int j = 0;
        double last = 0.0;
        for (; j < m; ++j) {
            double* wk = outer_w;
            tangent(Vo + (int64_t)j * Nu, wk);
            dots(Vo, Nu, j + 1, wk, h.data());
            vupdate(Vo, Nu, j + 1, h.data(), -1.0, wk);
            dots(Vo, Nu, j + 1, wk, h2.data());
            vupdate(Vo, Nu, j + 1, h2.data(), -1.0, wk);
            for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = h[i] + h2[i];
            const double hn = norm(wk);
            last = hn;
            if (j + 1 < m) H[(size_t)(j + 1) * m + j] = hn;
            if (!(hn > 1e-14 * std::fabs(H[(size_t)j * m + j]) + 1e-300)) { ++j; break; }
            if (j + 1 < m) lincomb(1.0 / hn, wk, 0.0, wk, Vo + (int64_t)(j + 1) * Nu);
            if (verbose && (j + 1) % 10 == 0) fprintf(stderr, "[pa] floquet arnoldi %d/%d\n", j + 1, m);
        }
        const int kk = std::min(j, m);
        std::vector<std::complex<double>> Hc((size_t)kk * kk), ev;
        for (int r = 0; r < kk; ++r)
            for (int c = 0; c < kk; ++c) Hc[(size_t)r * kk + c] = H[(size_t)r * m + c];
        hess_eig(Hc, kk, ev);
        std::sort(ev.begin(), ev.end(), [](const std::complex<double>& a, const std::complex<double>& b) {
            return std::abs(a) > std::abs(b);
        });
        for (int i = 0; i < kk; ++i) { re[i] = ev[i].real(); im[i] = ev[i].imag(); }
        if (hsub) *hsub = last;
        return kk;
    }

    // Alg. 1: m fixed-point periods u0 <- u^(Nt)(u0)
    void fixed_point(int periods, double* res_out) override
    {
        double res = 0.0, qoi[2];
        for (int k = 0; k < periods; ++k) {
            primal_sweep(qoi, &res);
            copy(tu + (int64_t)Nt * Nu, u0);
            have_traj = false;   // the stored trajectory starts from the previous u0
            if (verbose) fprintf(stderr, "[pa] fixed-point period %d |R| = %.3e\n", k + 1, res);
        }
        if (res_out) *res_out = res;
    }

    // Gradient of j(u0) = 1/2 ||u^(Nt)(u0) - u0||^2 (Sec. 2.2 eq. opt-obj) on
    // the stored trajectory: the backward sweep started from lam^(Nt) = R =
    // u^(Nt) - u0 returns lam^(0) = Phi^T R, and dj/du0 = lam^(0) - R (eq.
    // funcl-grad-nosens-dirk).  R and g are device vectors; returns j.
    double periodicity_grad_dev(double* R, double* g)
    {
        if (!have_traj) raise(PA_ESTATE, "no trajectory (run pa_primal_period first)");
        lincomb(1.0, tu + (int64_t)Nt * Nu, -1.0, u0, R);
        adjoint(R, -1, g, nullptr);
        axpby(-1.0, R, 1.0, g);
        const double rn = norm(R);
        return 0.5 * rn * rn;
    }
    static constexpr int DS_MAXMEM = 32;
    double *ds_R = nullptr, *ds_g = nullptr, *ds_d = nullptr, *ds_u = nullptr, *ds_q = nullptr, *ds_S = nullptr,
           *ds_Y = nullptr;
    int ds_mem = -1;
    void ensure_descent(int memory)
    {
        if (!ds_R) {
            ds_R = dalloc<double>(Nu);
            ds_g = dalloc<double>(Nu);
            ds_d = dalloc<double>(Nu);
            ds_u = dalloc<double>(Nu);
            ds_q = dalloc<double>(Nu);
        }
        if (memory > ds_mem) {
            ds_S = dalloc<double>((int64_t)std::max(memory, 1) * Nu);
            ds_Y = dalloc<double>((int64_t)std::max(memory, 1) * Nu);
            ds_mem = memory;
        }
    }
    double periodicity_gradient(double* grad) override
    {
        ensure_descent(0);
        const double j = periodicity_grad_dev(ds_R, ds_g);
        if (grad) d2h(grad, ds_g, sizeof(double) * Nu);
        return j;
    }
    double dot1(const double* a, const double* b)
    {
        double v;
        dots(a, Nu, 1, b, &v);
        return v;
    }

    // Shooting as unconstrained minimisation of j(u0) (Sec. 2.2, the
    // gradient-based alternative to Alg. 1 and 2): steepest descent
    // (memory 0) or L-BFGS with `memory` correction pairs.  Every iterate
    // costs one backward sweep for its gradient.  The step u0 + alpha d is
    // accepted when its primal period succeeds and j falls by at least
    // 1e-4 alpha |g^T d| (alpha = 1, 1/2, ..., 1/2^15).  The L-BFGS direction
    // is the two-loop recursion over the stored pairs (s, y) = (step,
    // gradient change), newest first, with the initial matrix s^T y / y^T y I
    // of the newest pair; a pair enters only when s^T y > 0, and a direction
    // that is not downhill restarts from steepest descent.  With Phi = 0 the
    // unit steepest-descent step is one fixed-point period.
    void shoot_descent(double tol, int memory, int maxit, pa_shoot_report* rep) override
    {
        double t0 = now_ms();
        pa_shoot_report r{};
        cnt_newton = cnt_gmres = 0;
        auto finish = [&]() {
            r.stage_newton_its = (int32_t)cnt_newton;
            r.stage_gmres_its = cnt_gmres;
            r.ms = now_ms() - t0;
            if (rep) *rep = r;
        };
        ensure_descent(memory);
        double *R = ds_R, *g = ds_g, *d = ds_d, *us = ds_u, *q = ds_q;
        auto S = [&](int i) { return ds_S + (int64_t)i * Nu; };
        auto Y = [&](int i) { return ds_Y + (int64_t)i * Nu; };
        std::vector<double> rho(std::max(memory, 1)), al(std::max(memory, 1));
        int npair = 0, newest = -1;
        double qoi[2], res;
        primal_sweep(qoi, &res);
        ++r.primal_sweeps;
        r.res0 = r.res = res;
        double j = periodicity_grad_dev(R, g);
        ++r.krylov_its;
        while (!(res <= tol)) {
            if (r.newton_its >= maxit) {
                finish();
                raise(PA_ENOCONV, "descent shooting did not converge: |R| = %.3e after %d iterations", res,
                      r.newton_its);
            }
            if (npair == 0) {
                lincomb(-1.0, g, 0.0, g, d);
            } else {
                copy(g, q);
                for (int k = 0; k < npair; ++k) {   // newest to oldest
                    const int i = (newest - k + memory) % memory;
                    al[i] = rho[i] * dot1(S(i), q);
                    axpby(-al[i], Y(i), 1.0, q);
                }
                const double gam = dot1(S(newest), Y(newest)) / dot1(Y(newest), Y(newest));
                lincomb(-gam, q, 0.0, q, d);   // d = -H0 q; the second loop acts on -d
                for (int k = npair - 1; k >= 0; --k) {   // oldest to newest
                    const int i = (newest - k + memory) % memory;
                    const double beta = -rho[i] * dot1(Y(i), d);
                    axpby(-(al[i] - beta), S(i), 1.0, d);
                }
            }
            double gd = dot1(g, d);
            if (!(gd < 0.0)) {
                npair = 0;
                newest = -1;
                lincomb(-1.0, g, 0.0, g, d);
                gd = dot1(g, d);
            }
            copy(u0, us);
            double alpha = 1.0, rnew = 0.0;
            bool ok = false;
            for (int trial = 0; trial < 16; ++trial, alpha *= 0.5) {
                lincomb(1.0, us, alpha, d, u0);
                try {
                    primal_sweep(qoi, &rnew);
                    ++r.primal_sweeps;
                    ok = 0.5 * rnew * rnew <= j + 1e-4 * alpha * gd;
                } catch (const PaError& e) {
                    if (e.code != PA_ENOCONV && e.code != PA_ENUMERIC) throw;
                    ++r.primal_sweeps;
                    ok = false;
                }
                if (ok) break;
            }
            if (!ok) {
                copy(us, u0);
                primal_sweep(qoi, &res);
                ++r.primal_sweeps;
                finish();
                raise(PA_ENOCONV, "descent shooting line search failed at |R| = %.3e", res);
            }
            const int slot = memory > 0 ? (newest + 1) % memory : 0;
            if (memory > 0) {
                lincomb(alpha, d, 0.0, d, S(slot));
                lincomb(-1.0, g, 0.0, g, Y(slot));
            }
            j = periodicity_grad_dev(R, g);
            ++r.krylov_its;
            res = rnew;
            r.res = res;
            ++r.newton_its;
            if (memory > 0) {
                axpby(1.0, g, 1.0, Y(slot));   // y = g_new - g_old
                const double sy = dot1(S(slot), Y(slot));
                if (sy > 0.0) {
                    rho[slot] = 1.0 / sy;
                    newest = slot;
                    npair = std::min(npair + 1, memory);
                } else if (npair == memory) {
                    --npair;   // the slot held the oldest pair, now overwritten
                }
            }
            if (verbose)
                fprintf(stderr, "[pa] descent it %d alpha %.3g |R| = %.3e  %.1f s\n", r.newton_its, alpha, res,
                        (now_ms() - t0) / 1e3);
        }
        finish();
    }

    // Outer matrix-free GMRES on (Phi - I) (tangent_op) or (Phi^T - I), zero
    // initial guess, no restart; rhs copied first, solution written to wf.
    // The sweeps' work vectors are disjoint from the outer buffers.
    void outer_gmres(bool tangent_op, const double* rhs, double rtol, int32_t& its_acc)
    {
        copy(rhs, outer_rhs);
        int nmv = 0;
        double t0 = now_ms();
        auto A = [&](const double* v, double* out) {
            if (tangent_op) tangent(v, out);
            else adjoint(v, -1, out, nullptr);
            axpby(-1.0, v, 1.0, out);
            if (verbose && (++nmv % 10) == 0)
                fprintf(stderr, "[pa]   %s sweeps %d  %.1f s\n", tangent_op ? "tangent" : "adjoint", nmv,
                        (now_ms() - t0) / 1e3);
        };
        double rr;
        int its = gmres(A, nullptr, outer_rhs, outer_x, rtol, max_kry, max_kry, Vo, outer_w, outer_z, &rr, false);
        its_acc += its;
        last_outer_rel = rr;
        copy(outer_x, wf);
    }
    double *outer_x = nullptr, *outer_w = nullptr, *outer_z = nullptr, *outer_rhs = nullptr, *lam_buf = nullptr;
    double *nk_delta = nullptr, *nk_save = nullptr;
    double *gm_b = nullptr, *gm_y = nullptr;
    double last_outer_rel = 0;

    // Outer matrix-free GMRES on (Phi^T - I) for R right-hand sides in
    // lockstep (no restart, zero initial guess): every iteration applies one
    // backward sweep carrying the current basis vector of each unconverged
    // system; Gram-Schmidt (two passes) and Givens rotations per system as in
    // gmres().  Solutions to outm (R vectors at stride Nu).
    double *VoM = nullptr, *stgX = nullptr, *stgY = nullptr, *outm = nullptr, *brhs = nullptr;
    void outer_adjoint_multi(int R, const double* rhs, double rtol, int32_t* its, double* rel)
    {
        outer_multi(false, R, rhs, rtol, its, rel);
    }
    // <V_c, w> and w += sign sum_c h_c V_c over more columns than one
    // multi-dot launch holds (chunks of the partials buffer's width)
    void dots_n(const double* V0, int ncols, const double* w, double* h)
    {
        const int ch = std::max(restart, max_kry);
        for (int c = 0; c < ncols; c += ch) dots(V0 + (int64_t)c * Nu, Nu, std::min(ch, ncols - c), w, h + c);
    }
    void vupdate_n(const double* V0, int ncols, const double* h, double sign, double* w)
    {
        const int ch = std::max(restart, max_kry);
        for (int c = 0; c < ncols; c += ch) vupdate(V0 + (int64_t)c * Nu, Nu, std::min(ch, ncols - c), h + c, sign, w);
    }

    // Block GMRES on (Phi - I) or (Phi^T - I) for R right-hand sides that
    // share one Krylov space (the multiple-right-hand-side setting of Sec.
    // 3.2: the operator is fixed, only b varies).  Zero initial guess, no
    // restart, block size R, at most max_krylov block iterations:
    //  - V_0 S_0 = B by Gram-Schmidt with a second pass;
    //  - iteration j applies one sweep carrying the R vectors of block j,
    //    orthogonalises each result against every basis vector so far (two
    //    passes) and normalises it, which gives column jR + l of the banded
    //    block Hessenberg matrix (R subdiagonals);
    //  - each new column is reduced by the earlier Givens rotations and R new
    //    ones; the same rotations act on the R columns of E_1 S_0, whose rows
    //    (j+1)R .. (j+2)R-1 then hold every system's residual.
    // Returns false, leaving outm untouched, when the right-hand sides or a
    // new block are numerically dependent (the caller then solves the
    // systems in separate spaces).
    bool outer_block(bool tangent_op, int R, const double* rhs, double rtol, int32_t* its, double* rel)
    {
        ensure_multi();
        if (!VoM) VoM = dalloc<double>((int64_t)GM_RMAX * (max_kry + 1) * Nu);
        const int kmax = std::min(max_kry, GM_RMAX * (max_kry + 1) / R - 1);
        const int nrow = (kmax + 1) * R, ncol = kmax * R;
        auto V = [&](int c) { return VoM + (int64_t)c * Nu; };
        std::vector<double> Hc((size_t)nrow * ncol, 0.0), G((size_t)nrow * R, 0.0);
        std::vector<double> h(nrow), h2(nrow), col(nrow), bn(R), res(R);
        struct Rot { int a, b; double c, s; };
        std::vector<Rot> rots;
        for (int q = 0; q < R; ++q) {
            its[q] = 0;
            rel[q] = 0.0;
            bn[q] = norm(rhs + (int64_t)q * Nu);
            if (!(bn[q] > 0.0)) return false;
        }
        for (int l = 0; l < R; ++l) {
            double* w = V(l);
            copy(rhs + (int64_t)l * Nu, w);
            if (l > 0) {
                dots_n(V(0), l, w, h.data());
                vupdate_n(V(0), l, h.data(), -1.0, w);
                dots_n(V(0), l, w, h2.data());
                vupdate_n(V(0), l, h2.data(), -1.0, w);
                for (int i = 0; i < l; ++i) G[(size_t)i * R + l] = h[i] + h2[i];
            }
            const double nr = norm(w);
            if (!(nr > 1e-10 * bn[l])) return false;
            G[(size_t)l * R + l] = nr;
            lincomb(1.0 / nr, w, 0.0, w, w);
        }
        const int fq[GM_RMAX] = { -1, -1, -1, -1, -1, -1, -1, -1 };
        double t0 = now_ms();
        int k = 0;
        bool conv = false;
        for (int j = 0; j < kmax && !conv; ++j) {
            HIPCHK(hipMemcpyAsync(stgX, V(j * R), sizeof(double) * R * Nu, hipMemcpyDeviceToDevice, st));
            if (tangent_op) tangent_multi(R, stgX, fq, stgY, nullptr);
            else adjoint_multi(R, stgX, fq, stgY, nullptr);
            for (int q = 0; q < R; ++q) ++its[q];
            for (int l = 0; l < R; ++l) {
                const int c = j * R + l, nc = c + R;   // column of H; basis vectors before the new one
                double* w = stgY + (int64_t)l * Nu;
                axpby(-1.0, stgX + (int64_t)l * Nu, 1.0, w);   // (Phi - I) v or (Phi^T - I) v
                dots_n(V(0), nc, w, h.data());
                vupdate_n(V(0), nc, h.data(), -1.0, w);
                dots_n(V(0), nc, w, h2.data());
                vupdate_n(V(0), nc, h2.data(), -1.0, w);
                const double hn = norm(w);
                if (!std::isfinite(hn)) raise(PA_ENUMERIC, "NaN in block GMRES");
                double cn = hn * hn;
                for (int i = 0; i < nc; ++i) {
                    col[i] = h[i] + h2[i];
                    cn += col[i] * col[i];
                }
                col[nc] = hn;
                if (!(hn > 1e-13 * std::sqrt(cn))) return false;
                lincomb(1.0 / hn, w, 0.0, w, V(nc));
                for (const Rot& r : rots) {
                    const double a = col[r.a], b = col[r.b];
                    col[r.a] = r.c * a + r.s * b;
                    col[r.b] = -r.s * a + r.c * b;
                }
                for (int i = c + 1; i <= nc; ++i) {
                    const double a = col[c], b = col[i];
                    const double rr = std::hypot(a, b);
                    if (rr == 0.0) continue;
                    const Rot r{ c, i, a / rr, b / rr };
                    col[c] = rr;
                    col[i] = 0.0;
                    for (int q = 0; q < R; ++q) {
                        const double ga = G[(size_t)c * R + q], gb = G[(size_t)i * R + q];
                        G[(size_t)c * R + q] = r.c * ga + r.s * gb;
                        G[(size_t)i * R + q] = -r.s * ga + r.c * gb;
                    }
                    rots.push_back(r);
                }
                for (int i = 0; i <= c; ++i) Hc[(size_t)i * ncol + c] = col[i];
            }
            k = j + 1;
            conv = true;
            for (int q = 0; q < R; ++q) {
                double s2 = 0.0;
                for (int i = k * R; i < (k + 1) * R; ++i) s2 += G[(size_t)i * R + q] * G[(size_t)i * R + q];
                res[q] = std::sqrt(s2);
                conv = conv && res[q] <= rtol * bn[q];
            }
            if (verbose && k % 10 == 0)
                fprintf(stderr, "[pa]   block %s sweeps %d (%d systems)  %.1f s\n", tangent_op ? "tangent" : "adjoint",
                        k, R, (now_ms() - t0) / 1e3);
        }
        const int n = k * R;
        std::vector<double> y(std::max(n, 1));
        for (int q = 0; q < R; ++q) {
            for (int i = n - 1; i >= 0; --i) {
                double t = G[(size_t)i * R + q];
                for (int p2 = i + 1; p2 < n; ++p2) t -= Hc[(size_t)i * ncol + p2] * y[p2];
                y[i] = t / Hc[(size_t)i * ncol + i];
            }
            zero(outm + (int64_t)q * Nu);
            if (n > 0) vupdate_n(V(0), n, y.data(), 1.0, outm + (int64_t)q * Nu);
            rel[q] = res[q] / bn[q];
        }
        return true;
    }

    // as above on (Phi - I) with tangent sweeps (tangent_op) or (Phi^T - I)
    void outer_multi(bool tangent_op, int R, const double* rhs, double rtol, int32_t* its, double* rel)
    {
        if (cfg.block_krylov && R > 1 && outer_block(tangent_op, R, rhs, rtol, its, rel)) return;
        ensure_multi();
        if (!VoM) VoM = dalloc<double>((int64_t)GM_RMAX * (max_kry + 1) * Nu);
        const int m = max_kry;
        struct Sys {
            std::vector<double> H, cs, sn, g, h, h2;
            double bn = 0, res = 0;
            int j = 0;
            bool active = true;
        };
        std::vector<Sys> S(R);
        auto Vb = [&](int r) { return VoM + (int64_t)r * (m + 1) * Nu; };
        for (int r = 0; r < R; ++r) {
            Sys& y = S[r];
            y.H.assign((m + 1) * m, 0.0); y.cs.assign(m, 0.0); y.sn.assign(m, 0.0); y.g.assign(m + 1, 0.0);
            y.h.assign(m + 2, 0.0); y.h2.assign(m + 2, 0.0);
            y.bn = norm(rhs + r * Nu);
            y.res = y.bn;
            y.g[0] = y.bn;
            y.active = y.bn > 0.0;
            its[r] = 0;
            if (y.active) lincomb(1.0 / y.bn, rhs + r * Nu, 0.0, rhs + r * Nu, Vb(r));
        }
        double t0 = now_ms();
        int nmv = 0;
        const int fq[GM_RMAX] = { -1, -1, -1, -1, -1, -1, -1, -1 };
        for (;;) {
            int act[GM_RMAX], na = 0;
            for (int r = 0; r < R; ++r)
                if (S[r].active) act[na++] = r;
            if (na == 0) break;
            for (int a = 0; a < na; ++a) copy(Vb(act[a]) + (int64_t)S[act[a]].j * Nu, stgX + a * Nu);
            if (tangent_op) tangent_multi(na, stgX, fq, stgY, nullptr);
            else adjoint_multi(na, stgX, fq, stgY, nullptr);
            ++nmv;
            if (verbose && nmv % 10 == 0)
                fprintf(stderr, "[pa]   %s sweeps %d (%d systems)  %.1f s\n", tangent_op ? "tangent" : "adjoint", nmv,
                        na, (now_ms() - t0) / 1e3);
            for (int a = 0; a < na; ++a) {
                const int r = act[a];
                Sys& y = S[r];
                const int j = y.j;
                double* wk = stgY + a * Nu;
                axpby(-1.0, stgX + a * Nu, 1.0, wk);   // (Phi - I) v or (Phi^T - I) v
                ++its[r];
                dots(Vb(r), Nu, j + 1, wk, y.h.data());
                vupdate(Vb(r), Nu, j + 1, y.h.data(), -1.0, wk);
                const int nb = (int)mdot_blocks(Nu);
                k_mdot_part<<<dim3(nb, mdot_chunks(j + 2)), MD_THREADS, 0, st>>>(Vb(r), Nu, j + 1, 1, wk, Nu, part, nullptr);
                k_mdot_fin<<<1, MD_THREADS, 0, st>>>(part, nb, j + 2, hdev);
                LAUNCHCHK();
                HIPCHK(hipMemcpyAsync(y.h2.data(), hdev, sizeof(double) * (j + 2), hipMemcpyDeviceToHost, st));
                HIPCHK(hipStreamSynchronize(st));
                double ww = y.h2[j + 1], corr = 0.0;
                for (int i = 0; i <= j; ++i) corr += y.h2[i] * y.h2[i];
                vupdate(Vb(r), Nu, j + 1, y.h2.data(), -1.0, wk);
                for (int i = 0; i <= j; ++i) y.H[i * m + j] = y.h[i] + y.h2[i];
                double hn = std::sqrt(std::max(ww - corr, 0.0));
                if (!std::isfinite(hn)) raise(PA_ENUMERIC, "NaN in GMRES");
                y.H[(j + 1) * m + j] = hn;
                for (int i = 0; i < j; ++i) {
                    double p = y.H[i * m + j], q = y.H[(i + 1) * m + j];
                    y.H[i * m + j] = y.cs[i] * p + y.sn[i] * q;
                    y.H[(i + 1) * m + j] = -y.sn[i] * p + y.cs[i] * q;
                }
                double p = y.H[j * m + j], q = y.H[(j + 1) * m + j];
                double rr = std::sqrt(p * p + q * q);
                y.cs[j] = p / rr;
                y.sn[j] = q / rr;
                y.H[j * m + j] = rr;
                y.H[(j + 1) * m + j] = 0.0;
                y.g[j + 1] = -y.sn[j] * y.g[j];
                y.g[j] = y.cs[j] * y.g[j];
                y.res = std::fabs(y.g[j + 1]);
                y.j = j + 1;
                const bool stop = y.res <= rtol * y.bn || hn == 0.0 || y.j >= m;
                if (!stop) lincomb(1.0 / hn, wk, 0.0, wk, Vb(r) + (int64_t)(j + 1) * Nu);
                else y.active = false;
            }
        }
        for (int r = 0; r < R; ++r) {
            Sys& y = S[r];
            const int k = y.j;
            std::vector<double> c(std::max(k, 1), 0.0);
            for (int i = k - 1; i >= 0; --i) {
                double t = y.g[i];
                for (int q = i + 1; q < k; ++q) t -= y.H[i * m + q] * c[q];
                c[i] = t / y.H[i * m + i];
            }
            zero(outm + r * Nu);
            if (k > 0) vupdate(Vb(r), Nu, k, c.data(), 1.0, outm + r * Nu);
            rel[r] = y.bn > 0.0 ? y.res / y.bn : 0.0;
        }
    }

    // Direct (tangent) gradient, Sec. 2.2 with the parameter forcing: for the
    // three parameters together, the forced tangent sweeps from zero give
    // s_k, the periodic tangents solve (Phi - I) du0_k = -s_k, and one forced
    // sweep from du0_k accumulates dJ_q/dmu_k.  Independent of the adjoint.
    void tangent_gradient(double rtol, double dJ[6], int32_t its_out[3]) override
    {
        if (!have_traj) raise(PA_ESTATE, "no trajectory (run pa_primal_period or pa_shoot first)");
        ensure_multi();
        const int dirs[3] = { 0, 1, 2 };
        zero(stgX, 3 * Nu);
        tangent_multi(3, stgX, dirs, brhs, nullptr);
        for (int k = 0; k < 3; ++k) axpby(-1.0, brhs + k * Nu, 0.0, brhs + k * Nu);
        int32_t its[3];
        double rel[3];
        outer_multi(true, 3, brhs, rtol, its, rel);
        HIPCHK(hipMemcpyAsync(stgX, outm, sizeof(double) * 3 * Nu, hipMemcpyDeviceToDevice, st));
        double dq[6];
        tangent_multi(3, stgX, dirs, stgY, dq);
        for (int k = 0; k < 3; ++k) {
            dJ[k] = dq[2 * k];
            dJ[3 + k] = dq[2 * k + 1];
            if (its_out) its_out[k] = its[k];
        }
        if (verbose)
            fprintf(stderr, "[pa] tangent gradient: %d / %d / %d krylov its, rel res %.1e / %.1e / %.1e\n", its[0],
                    its[1], its[2], rel[0], rel[1], rel[2]);
    }

    void adjoint_gradient(double rtol, double qoi[2], double dJ[6], pa_adjoint_report* rep) override
    {
        if (!have_traj) raise(PA_ESTATE, "no trajectory (run pa_primal_period or pa_shoot first)");
        double t0 = now_ms();
        int64_t g0 = cnt_gmres;
        pa_adjoint_report r{};
        // both QoIs in lockstep: every backward sweep carries one right-hand
        // side per QoI (g_F sweeps, the Krylov sweeps, the final sweeps)
        ensure_multi();
        const int fq[2] = { 0, 1 };
        double grad[6];
        zero(stgX, 2 * Nu);
        adjoint_multi(2, stgX, fq, brhs, grad);          // g_F of both QoIs from zero
        r.sweeps += 1;
        r.rhs_sweeps += 2;
        axpby(-1.0, brhs, 0.0, brhs);                    // b = -g_F  (dF/du^(Nt) = 0)
        axpby(-1.0, brhs + Nu, 0.0, brhs + Nu);
        int32_t its[2];
        double rel[2];
        outer_adjoint_multi(2, brhs, rtol, its, rel);
        for (int q = 0; q < 2; ++q) {
            r.krylov_its[q] = its[q];
            r.rel_res[q] = rel[q];
        }
        r.sweeps += std::max(its[0], its[1]);
        r.rhs_sweeps += its[0] + its[1];
        if (verbose)
            fprintf(stderr, "[pa] adjoint (2 QoIs, %s): %d / %d krylov its, rel res %.2e / %.2e, %.1f s\n",
                    cfg.block_krylov ? "one block space" : "lockstep", its[0], its[1], rel[0], rel[1],
                    (now_ms() - t0) / 1e3);
        HIPCHK(hipMemcpyAsync(stgX, outm, sizeof(double) * 2 * Nu, hipMemcpyDeviceToDevice, st));
        adjoint_multi(2, stgX, fq, stgY, grad);
        r.sweeps += 1;
        r.rhs_sweeps += 2;
        for (int k = 0; k < 6; ++k) dJ[k] = grad[k];
        if (qoi) {
            // time-averaged QoIs of the stored trajectory
            std::vector<double> h((size_t)nst * std::max(nwall, 1) * 2);
            d2h(h.data(), qh, sizeof(double) * h.size());
            double J0 = 0, J1 = 0;
            for (int s = 0; s < nst; ++s) {
                double f0 = 0, f1 = 0;
                for (int w = 0; w < nwall; ++w) { f0 += h[((size_t)s * nwall + w) * 2]; f1 += h[((size_t)s * nwall + w) * 2 + 1]; }
                J0 += dt * rk.b[s % 3] * f0 / cfg.T;
                J1 += dt * rk.b[s % 3] * f1 / cfg.T;
            }
            qoi[0] = J0;
            qoi[1] = J1;
        }
        r.stage_gmres_its = cnt_gmres - g0;
        r.ms = now_ms() - t0;
        if (rep) *rep = r;
    }

    // ---------------------------------------------------------------- host-vector wrappers
    void tangent_sweep_h(const double* v, double* out) override
    {
        h2d(wd, v, sizeof(double) * Nu);
        tangent(wd, wf);
        d2h(out, wf, sizeof(double) * Nu);
    }
    void adjoint_sweep_h(const double* lamh, int fq, double* lam0, double* grad) override
    {
        h2d(wd, lamh, sizeof(double) * Nu);
        adjoint(wd, fq, wf, grad);
        d2h(lam0, wf, sizeof(double) * Nu);
    }

    // ---------------------------------------------------------------- debug entry points
    void dbg_gbar(int n, int i, double* out, bool deriv) override
    {
        check_stage(n, i);
        if (deriv) d2h(out, dgbs(n, i), sizeof(double) * 3 * nn);
        else d2h(out, gbs(n, i), sizeof(double) * nn);
    }
    void dbg_residual(int n, int i, const double* u, double* r, bool dmu) override
    {
        check_stage(n, i);
        h2d(wd, u, sizeof(double) * Nu);
        if (dmu) {
            dr_dmu(n, i, wd, drm);
            HIPCHK(hipStreamSynchronize(st));
            d2h(r, drm, sizeof(double) * 3 * Nu);
        } else {
            residual(n, i, wd, wf);
            HIPCHK(hipStreamSynchronize(st));
            d2h(r, wf, sizeof(double) * Nu);
        }
    }
    void dbg_jacobian(int n, int i, const double* u, double* blk) override
    {
        check_stage(n, i);
        h2d(wd, u, sizeof(double) * Nu);
        jacobian(n, i, wd, Jtmp);
        d2h(blk, Jtmp, sizeof(double) * Jsz);
        have_traj = false;
    }
    void dbg_qoi(int n, int i, const double* u, double f[2], double* dfdu, double* dfdmu) override
    {
        check_stage(n, i);
        h2d(wd, u, sizeof(double) * Nu);
        double fv[2] = { 0, 0 };
        if (dfdu) {
            for (int q = 0; q < 2; ++q) {
                qoi_grad(n, i, wd, q, wf, qtmp);
                HIPCHK(hipStreamSynchronize(st));
                d2h(dfdu + (int64_t)q * Nu, wf, sizeof(double) * Nu);
            }
        }
        double fm[6];
        qoi_dmu(n, i, wd, fm, fv);
        if (f) { f[0] = fv[0]; f[1] = fv[1]; }
        if (dfdmu) std::memcpy(dfdmu, fm, sizeof fm);
    }
    void dbg_bsr_apply(const double* blk, double alpha, double beta, int tr, const double* x, double* y) override
    {
        h2d(Jtmp, blk, sizeof(double) * Jsz);
        h2d(wd, x, sizeof(double) * Nu);
        bsr(Jtmp, alpha, beta, tr, wd, wf);
        HIPCHK(hipStreamSynchronize(st));
        d2h(y, wf, sizeof(double) * Nu);
        have_traj = false;
    }
    void dbg_blockinv(const double* blk, double adt, double* out) override
    {
        h2d(Jtmp, blk, sizeof(double) * Jsz);
        HIPCHK(hipMemsetAsync(dstatus, 0, sizeof(int), st));
        prepare_ops(Jtmp, adt, 0);
        int stt = 0;
        HIPCHK(hipMemcpyAsync(&stt, dstatus, sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (stt) raise(PA_ENUMERIC, "singular diagonal block");
        d2h(out, tAi, sizeof(double) * Isz);
        have_traj = false;
    }
    int dbg_stage_solve(const double* blk, double adt, int tr, const double* rhs, double* x) override
    {
        h2d(Jtmp, blk, sizeof(double) * Jsz);
        prepare_ops(Jtmp, adt, 0);
        h2d(wd, rhs, sizeof(double) * Nu);
        StageOps op = ops(0);
        op.aii = adt;
        int its = stage_solve(op, tr, wd, wc);
        HIPCHK(hipStreamSynchronize(st));
        d2h(x, wc, sizeof(double) * Nu);
        have_traj = false;
        return its;
    }
    int done_stages = 0;   // stages completed by the last (possibly failed) primal sweep
    void dbg_traj(int which, int n, int i, double* out) override
    {
        // stages of a sweep that stopped early stay readable (diagnostics)
        int need = which == 2 ? 3 * n : (n - 1) * 3 + i;
        if (!have_traj && need > done_stages) raise(PA_ESTATE, "no trajectory");
        const double* src;
        if (which == 2) {
            if (n < 0 || n > Nt) raise(PA_EINVAL, "bad step");
            src = tu + (int64_t)n * Nu;
        } else {
            if (n < 1 || n > Nt || i < 1 || i > 3) raise(PA_EINVAL, "bad stage");
            int s = (n - 1) * 3 + (i - 1);
            src = which == 0 ? stU(s) : stK(s);
        }
        d2h(out, src, sizeof(double) * Nu);
    }
    // reps launches of the apply that carries R right-hand sides at once
    // (x = R zero vectors: the timing does not depend on the values)
    double bench_spmv_m(int reps, int tr, int R) override
    {
        if (!have_traj) raise(PA_ESTATE, "no trajectory");
        if (R < 1 || R > GM_RMAX) raise(PA_EINVAL, "right-hand sides must be 1..%d", GM_RMAX);
        if (reps < 1) raise(PA_EINVAL, "reps must be positive");
        ensure_multi();
        zero(lamm, (int64_t)R * Nu);
        hipEvent_t a, b;
        HIPCHK(hipEventCreate(&a));
        HIPCHK(hipEventCreate(&b));
        const double* Ah = ops(0).Ah;
        ahat_m(Ah, tr, R, lamm, Nu, rhsm, Nu);
        HIPCHK(hipEventRecord(a, st));
        for (int r = 0; r < reps; ++r) ahat_m(Ah, tr, R, lamm, Nu, rhsm, Nu);
        HIPCHK(hipEventRecord(b, st));
        HIPCHK(hipEventSynchronize(b));
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, a, b));
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        return ms / reps;
    }
    double bench_spmv(int reps, int tr) override
    {
        if (!have_traj) raise(PA_ESTATE, "no trajectory");
        hipEvent_t a, b;
        HIPCHK(hipEventCreate(&a));
        HIPCHK(hipEventCreate(&b));
        const double* Ah = ops(0).Ah;
        ahat(Ah, tr, u0, wf);
        HIPCHK(hipEventRecord(a, st));
        for (int r = 0; r < reps; ++r) ahat(Ah, tr, u0, wf);
        HIPCHK(hipEventRecord(b, st));
        HIPCHK(hipEventSynchronize(b));
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, a, b));
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        return ms / reps;
    }

    void tuning(int32_t* q, double us[3]) override
    {
        if (q) *q = fwd_q;
        if (us) for (int k = 0; k < 3; ++k) us[k] = fwd_tune_us[k];
    }
    double bench_spmv_lo(int reps, int tr) override
    {
        if (!have_traj) raise(PA_ESTATE, "no trajectory");
        if (pmode == PA_PREC_FP64) raise(PA_ESTATE, "context has no low-precision operator (precision FP64)");
        hipEvent_t a, b;
        HIPCHK(hipEventCreate(&a));
        HIPCHK(hipEventCreate(&b));
        const void* Al = ops(0).Al;
        k_scale_to_f32<<<grid1(Nu), 256, 0, st>>>(1.0, u0, r32, Nu);
        ahat_lo(Al, tr, r32, w32);
        HIPCHK(hipEventRecord(a, st));
        for (int r = 0; r < reps; ++r) ahat_lo(Al, tr, r32, w32);
        HIPCHK(hipEventRecord(b, st));
        HIPCHK(hipEventSynchronize(b));
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, a, b));
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        return ms / reps;
    }

    // plain device-to-device copy of the first stage's stored operator
    // (a copy kernel of known size, used to calibrate traffic counters)
    double bench_copy(int reps, int64_t* bytes) override
    {
        if (nst < 2) raise(PA_EINVAL, "needs at least two stored stages");
        const size_t nb = sizeof(double) * 3 * (size_t)Isz;
        hipEvent_t a, b;
        HIPCHK(hipEventCreate(&a));
        HIPCHK(hipEventCreate(&b));
        HIPCHK(hipMemcpyAsync(tAh + 3 * Isz, tAh, nb, hipMemcpyDeviceToDevice, st));
        HIPCHK(hipEventRecord(a, st));
        for (int r = 0; r < reps; ++r) HIPCHK(hipMemcpyAsync(tAh + 3 * Isz, tAh, nb, hipMemcpyDeviceToDevice, st));
        HIPCHK(hipEventRecord(b, st));
        HIPCHK(hipEventSynchronize(b));
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, a, b));
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        have_traj = false;
        if (bytes) *bytes = (int64_t)nb;
        return ms / reps;
    }

    int64_t num_dofs() const override { return Nu; }
    int32_t num_elems() const override { return Ne; }
    int32_t block_size() const override { return B; }
    int64_t device_bytes() const override { return bytes; }
    void get_mesh(int32_t* a, int32_t* b, int8_t* c, double* d) const override
    {
        if (a) std::memcpy(a, ev.data(), sizeof(int32_t) * ev.size());
        if (b) std::memcpy(b, enb.data(), sizeof(int32_t) * enb.size());
        if (c) std::memcpy(c, etw.data(), sizeof(int8_t) * etw.size());
        if (d) std::memcpy(d, vxy.data(), sizeof(double) * vxy.size());
    }
};

pa_status guard(pa_ctx* c, const std::function<void()>& f)
{
    if (!c) return PA_EINVAL;
    try {
        f();
        return PA_OK;
    } catch (const PaError& e) {
        c->err = e.msg;
        return e.code;
    } catch (const std::exception& e) {
        c->err = e.what();
        return PA_EDEVICE;
    }
}

}  // namespace

// ------------------------------------------------------------------ C ABI
extern "C" {

void pa_default_config(pa_config* c)
{
    std::memset(c, 0, sizeof *c);
    c->Nr = 8; c->Nth = 24; c->p = 1; c->Nt = 20;
    c->r_far = 10.0; c->stretch = 1.3;
    c->mach = 0.2; c->re = 1000.0; c->gamma = 1.4; c->pr = 0.72;
    c->T = 1.0; c->r_blend0 = 2.0; c->r_blend1 = 8.0;
    c->wall_is_farfield = 0;
    c->gmres_restart = 30; c->lin_rtol = 1e-10;
    c->newton_atol = 1e-10; c->newton_maxit = 20;
    c->max_krylov = 100;
    c->precision = PA_PREC_FP64;
    c->autotune = 0;
    c->block_krylov = 0;
    c->device = 0;
    c->wg_solve = 0;
    c->lin_guess = 0;
    c->graph = 0;
}

static thread_local std::string g_create_err;

pa_status pa_create(const pa_config* cfg, pa_ctx** out)
{
    if (!out) return PA_EINVAL;
    *out = nullptr;
    if (!cfg || cfg->Nr < 1 || cfg->Nth < 3 || cfg->p < 1 || cfg->p > 3 || cfg->Nt < 1 || cfg->gmres_restart < 1 ||
        cfg->gmres_restart > 64 || cfg->max_krylov < 1 || cfg->max_krylov > 126 || !(cfg->r_far > 1.0) ||
        !(cfg->stretch > 0.0) || !(cfg->T > 0.0) || cfg->precision < PA_PREC_FP64 || cfg->precision > PA_PREC_BF16 ||
        cfg->wg_solve < -1 || cfg->wg_solve > 1 || cfg->lin_guess < 0 || cfg->lin_guess > 1 || cfg->graph < 0 ||
        cfg->graph > 1) {
        g_create_err = "invalid configuration";
        return PA_EINVAL;
    }
    if (cfg->graph == 1 && (cfg->gmres_restart % Solver<1>::GM_CHECK != 0 || cfg->precision != PA_PREC_FP64 || cfg->wg_solve != 0)) {
        g_create_err = "graph = 1 needs gmres_restart a multiple of 5, FP64 precision and wg_solve = 0";
        return PA_EINVAL;
    }
    if (cfg->wg_solve == 1) {
        const int64_t np_ = (int64_t)(cfg->p + 1) * (cfg->p + 2) / 2;
        const int64_t nu = 2LL * cfg->Nr * cfg->Nth * 4 * np_;
        if (nu > WG_MAXNU || cfg->gmres_restart > WG_MAXM) {
            g_create_err = "wg_solve = 1 needs N_u <= " + std::to_string(WG_MAXNU) + " and gmres_restart <= " +
                           std::to_string(WG_MAXM);
            return PA_EINVAL;
        }
    }
    try {
        pa_ctx* c = nullptr;
        switch (cfg->p) {
        case 1: c = new Solver<1>(*cfg); break;
        case 2: c = new Solver<2>(*cfg); break;
        default: c = new Solver<3>(*cfg); break;
        }
        *out = c;
        return PA_OK;
    } catch (const PaError& e) {
        g_create_err = e.msg;
        return e.code;
    } catch (const std::exception& e) {
        g_create_err = e.what();
        return PA_EDEVICE;
    }
}

void pa_destroy(pa_ctx* c) { delete c; }
const char* pa_last_error(const pa_ctx* c) { return c ? c->err.c_str() : g_create_err.c_str(); }
int64_t pa_num_dofs(const pa_ctx* c) { return c ? c->num_dofs() : -1; }

// host-only entry points of the small dense eigen-solvers (no device work)
pa_status pa_dbg_hess_eig(int32_t n, const double* H, double* re, double* im)
{
    try {
        if (n < 1 || n > 1024 || !H || !re || !im) raise(PA_EINVAL, "bad arguments");
        std::vector<std::complex<double>> Hc((size_t)n * n), ev;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) Hc[(size_t)i * n + j] = j >= i - 1 ? H[(size_t)i * n + j] : 0.0;
        hess_eig(Hc, n, ev);
        std::sort(ev.begin(), ev.end(), [](const std::complex<double>& a, const std::complex<double>& b) {
            return std::abs(a) > std::abs(b);
        });
        for (int i = 0; i < n; ++i) { re[i] = ev[i].real(); im[i] = ev[i].imag(); }
        return PA_OK;
    } catch (const PaError& e) {
        g_create_err = e.msg;
        return e.code;
    }
}
pa_status pa_dbg_sym_eig(int32_t n, const double* A, double* w, double* V)
{
    try {
        if (n < 1 || n > 1024 || !A || !w || !V) raise(PA_EINVAL, "bad arguments");
        std::vector<double> M(A, A + (size_t)n * n), lam, vec;
        sym_eig(M, n, lam, vec);
        std::copy(lam.begin(), lam.end(), w);
        std::copy(vec.begin(), vec.end(), V);
        return PA_OK;
    } catch (const PaError& e) {
        g_create_err = e.msg;
        return e.code;
    }
}
int32_t pa_num_elems(const pa_ctx* c) { return c ? c->num_elems() : -1; }
int32_t pa_block_size(const pa_ctx* c) { return c ? c->block_size() : -1; }
int64_t pa_device_bytes(const pa_ctx* c) { return c ? c->device_bytes() : -1; }

pa_status pa_get_mesh(const pa_ctx* c, int32_t* a, int32_t* b, int8_t* t, double* v)
{
    if (!c) return PA_EINVAL;
    c->get_mesh(a, b, t, v);
    return PA_OK;
}
pa_status pa_set_params(pa_ctx* c, const double mu[3])
{
    return guard(c, [&] { if (!mu) raise(PA_EINVAL, "null mu"); c->set_params(mu); });
}
pa_status pa_set_state(pa_ctx* c, const double* u0, int64_t n)
{
    return guard(c, [&] { if (!u0) raise(PA_EINVAL, "null state"); c->set_state(u0, n); });
}
pa_status pa_set_freestream(pa_ctx* c, const double* pert) { return guard(c, [&] { c->set_freestream(pert); }); }
pa_status pa_get_state(pa_ctx* c, int32_t which, double* out, int64_t n)
{
    return guard(c, [&] { if (!out) raise(PA_EINVAL, "null output"); c->get_state(which, out, n); });
}
pa_status pa_primal_period(pa_ctx* c, double qoi[2], double* res)
{
    return guard(c, [&] { c->primal_period(qoi, res); });
}
pa_status pa_ws_train(pa_ctx* c, const double* params, const double* states, int32_t S, const pa_ws_opts* o,
                      double* loss)
{
    return guard(c, [&] {
        if (!o) raise(PA_EINVAL, "no options");
        c->ws_train(params, states, S, *o, loss);
    });
}
pa_status pa_ws_predict(pa_ctx* c, const double mu[3])
{
    return guard(c, [&] {
        if (!mu) raise(PA_EINVAL, "no parameters");
        c->ws_predict(mu);
    });
}
pa_status pa_ws_shoot(pa_ctx* c, double tol, double eta, int32_t maxit, pa_shoot_report* rep, int32_t* fell_back)
{
    return guard(c, [&] {
        if (!(tol > 0) || !(eta > 0) || maxit < 1) raise(PA_EINVAL, "bad shooting options");
        c->ws_shoot(tol, eta, maxit, rep, fell_back);
    });
}
// ---- periodic-constrained optimisation (generalized reduced gradient) ----
// QP subproblem of the SQP step in n = 3 scaled variables:
//   minimise g.d + 1/2 d^T B d  subject to  a.d = -c,  lo <= d <= hi
// with B symmetric positive definite.  The minimiser lies in the relative
// interior of one face of the box, where it minimises the quadratic with the
// face's variables fixed at their bounds and the equality kept, so every
// face (each variable free, at its lower or at its upper bound: 27 faces)
// is solved and the feasible solution with the smallest objective is
// taken.  When no point of the box satisfies the equality, its target -c is
// first clamped to the range of a.d over the box (the least violation).
// Returns the equality multiplier in *lam (the constraint's Lagrange
// multiplier, sign convention g + B d = lam a + bound multipliers) and 0, or
// -1 when no face has a solution.
int qp3(const double B[9], const double g[3], const double a[3], double c, const double lo[3], const double hi[3],
        double d[3], double* lam)
{
    double amin = 0, amax = 0, anorm = 0;
    for (int i = 0; i < 3; ++i) {
        amin += a[i] > 0 ? a[i] * lo[i] : a[i] * hi[i];
        amax += a[i] > 0 ? a[i] * hi[i] : a[i] * lo[i];
        anorm = std::max(anorm, std::fabs(a[i]));
    }
    const bool has_eq = anorm > 0.0;         // a = 0: no equality (bounds only)
    const double target = has_eq ? std::min(std::max(-c, amin), amax) : 0.0;
    const double etol = 1e-9 * (1.0 + std::fabs(amin) + std::fabs(amax));   // equality tolerance
    double best = 1e300;
    int found = -1;
    for (int code = 0; code < 27; ++code) {
        int st[3] = { code % 3, (code / 3) % 3, code / 9 };   // 0 free, 1 lower, 2 upper
        double x[3] = { 0, 0, 0 };
        int fr[3], nf = 0;
        double fixed_a = 0.0, free_a = 0.0;
        for (int i = 0; i < 3; ++i) {
            if (st[i] == 1) x[i] = lo[i];
            else if (st[i] == 2) x[i] = hi[i];
            else fr[nf++] = i;
            if (st[i] != 0) fixed_a += a[i] * x[i];
            else free_a = std::max(free_a, std::fabs(a[i]));
        }
        // the equality constrains the free variables only when one of them enters it; otherwise the
        // fixed ones must satisfy it already
        const bool eq_row = has_eq && free_a > 0.0;
        if (has_eq && !eq_row && std::fabs(fixed_a - target) > etol) continue;
        // KKT of the free variables (with the equality when it binds them):
        // [Bff -aF; aF^T 0] [xF; l] = [-gF - Bfx x_fixed; t - a_fixed . x_fixed]
        const int m = nf + (eq_row ? 1 : 0);
        double K[4][5] = {};
        for (int r = 0; r < nf; ++r) {
            const int i = fr[r];
            double rhs = -g[i];
            for (int j = 0; j < 3; ++j)
                if (st[j] != 0) rhs -= B[i * 3 + j] * x[j];
            for (int q = 0; q < nf; ++q) K[r][q] = B[i * 3 + fr[q]];
            if (eq_row) K[r][nf] = -a[i];
            K[r][m] = rhs;
        }
        if (eq_row) {
            for (int q = 0; q < nf; ++q) K[nf][q] = a[fr[q]];
            K[nf][m] = target - fixed_a;
        }
        // Gauss-Jordan elimination with partial pivoting: K becomes diagonal, row k holding unknown k
        bool ok = true;
        for (int col = 0; col < m && ok; ++col) {
            int pv = col;
            for (int r = col + 1; r < m; ++r)
                if (std::fabs(K[r][col]) > std::fabs(K[pv][col])) pv = r;
            if (std::fabs(K[pv][col]) < 1e-300) { ok = false; break; }
            if (pv != col)
                for (int q = 0; q <= m; ++q) std::swap(K[col][q], K[pv][q]);
            for (int r = 0; r < m; ++r) {
                if (r == col) continue;
                const double f = K[r][col] / K[col][col];
                for (int q = col; q <= m; ++q) K[r][q] -= f * K[col][q];
            }
        }
        if (!ok) continue;
        const double l = eq_row ? K[nf][m] / K[nf][nf] : 0.0;
        for (int r = 0; r < nf; ++r) x[fr[r]] = K[r][m] / K[r][r];
        bool feas = true;
        for (int i = 0; i < 3; ++i) feas = feas && x[i] >= lo[i] - 1e-12 && x[i] <= hi[i] + 1e-12;
        if (has_eq) {
            double ax = 0.0;
            for (int i = 0; i < 3; ++i) ax += a[i] * x[i];
            feas = feas && std::fabs(ax - target) <= etol;
        }
        if (!feas) continue;
        double obj = 0.0;
        for (int i = 0; i < 3; ++i) {
            obj += g[i] * x[i];
            for (int j = 0; j < 3; ++j) obj += 0.5 * x[i] * B[i * 3 + j] * x[j];
        }
        if (obj < best) {
            best = obj;
            for (int i = 0; i < 3; ++i) d[i] = std::min(std::max(x[i], lo[i]), hi[i]);
            *lam = l;
            found = 0;
        }
    }
    if (found == 0 && has_eq) {
        // where the minimiser is degenerate (a vertex, or a face whose free variables the equality
        // does not bind, e.g. when the target was clamped) the face's multiplier need not carry the
        // right signs on the bound variables: take the valid multiplier nearest to it, from
        // w_i = (g + B d)_i = lam a_i on free variables, w_i - lam a_i >= 0 at a lower bound and
        // <= 0 at an upper bound
        double lmin = -1e300, lmax = 1e300;
        for (int i = 0; i < 3; ++i) {
            double w = g[i];
            for (int j = 0; j < 3; ++j) w += B[i * 3 + j] * d[j];
            const bool atl = d[i] <= lo[i] + 1e-12 * (1.0 + std::fabs(lo[i]));
            const bool atu = d[i] >= hi[i] - 1e-12 * (1.0 + std::fabs(hi[i]));
            if (a[i] == 0.0 || (atl && atu)) continue;
            const double q = w / a[i];
            if (!atl && !atu) { lmin = std::max(lmin, q); lmax = std::min(lmax, q); }
            else if (atl == (a[i] > 0)) lmax = std::min(lmax, q);   // lam a_i <= w_i
            else lmin = std::max(lmin, q);                          // lam a_i >= w_i
        }
        if (lmin <= lmax) *lam = std::min(std::max(*lam, lmin), lmax);
    }
    return found;
}

// Generalized reduced-gradient loop of Sec. 3.3 (eq. opt:disc2 reduced to
// eq. opt:disc1 on the manifold of periodic solutions): every evaluation at
// parameters mu shoots to the periodic orbit (Alg. 2, warm-started from the
// previous periodic state) and every accepted point takes both QoIs' periodic
// adjoint gradients (Alg. 3, Alg. 4).  The optimiser is a line-search SQP
// in variables scaled to the box [lo, hi]: QP steps (qp3) within a trust box,
// damped BFGS on the Hessian of the Lagrangian, l1 merit f + rho |c| with
// backtracking.  Minimises obj_sign J[obj] subject to J[con] = con_value
// (con < 0: no constraint).
void pa_ctx::optimize(const pa_opt_opts& o, double mu[3], pa_opt_report* rep)
{
    const double t0 = now_ms();
    pa_opt_report r{};
    if (rep) {
        r.mu_hist = rep->mu_hist;
        r.f_hist = rep->f_hist;
        r.c_hist = rep->c_hist;
        r.hist_cap = rep->hist_cap;
    }
    const bool constrained = o.con >= 0;
    double sc[3];
    for (int k = 0; k < 3; ++k) {
        if (!(o.hi[k] > o.lo[k])) raise(PA_EINVAL, "empty parameter box in variable %d", k);
        if (!(mu[k] >= o.lo[k] && mu[k] <= o.hi[k])) raise(PA_EINVAL, "start outside the parameter box");
        sc[k] = o.hi[k] - o.lo[k];
    }
    const int nu = (int)num_dofs();
    std::vector<double> uper(nu), ustart(nu);
    get_state(0, ustart.data(), nu);     // the first shooting starts from the context's current u0
    bool have_orbit = false;
    // one evaluation: periodic orbit at m, QoIs; gradient on request
    auto evaluate = [&](const double m[3], bool grad, double q[2], double dq[6]) -> bool {
        set_params(m);
        set_state(have_orbit ? uper.data() : ustart.data(), nu);
        pa_shoot_report sr{};
        try {
            shoot(o.shoot_tol, o.shoot_eta, o.shoot_maxit, &sr);
        } catch (const PaError& e) {
            if (e.code != PA_ENOCONV && e.code != PA_ENUMERIC) throw;
            r.shoots += 1;
            return false;
        }
        r.shoots += 1;
        r.newton_its += sr.newton_its;
        r.tangent_sweeps += sr.krylov_its;
        last_qois(q);
        if (grad) {
            pa_adjoint_report ar{};
            double qq[2];
            adjoint_gradient(o.adj_rtol, qq, dq, &ar);
            r.gradients += 1;
            r.adjoint_sweeps += ar.sweeps;
        }
        return true;
    };
    auto fval = [&](const double q[2]) { return o.obj_sign * q[o.obj]; };
    auto cval = [&](const double q[2]) { return constrained ? q[o.con] - o.con_value : 0.0; };
    double x[3], q[2], dq[6];
    for (int k = 0; k < 3; ++k) x[k] = (mu[k] - o.lo[k]) / sc[k];
    auto to_mu = [&](const double* y, double* m) { for (int k = 0; k < 3; ++k) m[k] = o.lo[k] + sc[k] * y[k]; };
    double m[3];
    to_mu(x, m);
    if (!evaluate(m, true, q, dq)) raise(PA_ENOCONV, "shooting failed at the starting parameters");
    get_state(0, uper.data(), nu);
    have_orbit = true;
    double f = fval(q), c = cval(q), g[3], a[3];
    for (int k = 0; k < 3; ++k) {
        g[k] = o.obj_sign * dq[3 * o.obj + k] * sc[k];
        a[k] = constrained ? dq[3 * o.con + k] * sc[k] : 0.0;
    }
    double B[9] = { 0 };
    {   // initial Hessian: identity scaled so that a unit gradient step moves a tenth of the box
        double gn = 0;
        for (int k = 0; k < 3; ++k) gn = std::max(gn, std::fabs(g[k]));
        const double s0 = gn > 0 ? 10.0 * gn : 1.0;
        for (int k = 0; k < 3; ++k) B[k * 4] = s0;
    }
    double lam = 0.0, rho = 0.0, delta = o.trust > 0 ? o.trust : 0.25;
    auto record = [&]() {
        const int k = r.iterations;
        if (k < r.hist_cap) {
            if (r.mu_hist) to_mu(x, r.mu_hist + 3 * k);
            if (r.f_hist) r.f_hist[k] = f;
            if (r.c_hist) r.c_hist[k] = c;
        }
    };
    auto kkt = [&]() {
        // projected gradient of the Lagrangian on the box (inf-norm, scaled variables)
        double e = 0;
        for (int k = 0; k < 3; ++k) {
            double gl = g[k] - lam * a[k];
            if (x[k] <= 1e-12 && gl > 0) gl = 0;
            if (x[k] >= 1 - 1e-12 && gl < 0) gl = 0;
            e = std::max(e, std::fabs(gl));
        }
        return e;
    };
    // multiplier estimate at the start: least squares g = lam a
    if (constrained) {
        double aa = 0, ga = 0;
        for (int k = 0; k < 3; ++k) { aa += a[k] * a[k]; ga += g[k] * a[k]; }
        lam = aa > 0 ? ga / aa : 0.0;
    }
    record();
    for (;;) {
        r.kkt = kkt();
        r.f = f;
        r.c = c;
        if (r.kkt <= o.tol_kkt && std::fabs(c) <= o.tol_c) { r.converged = 1; break; }
        if (r.iterations >= o.maxit) break;
        double lo3[3], hi3[3], d[3], lq = 0.0;
        for (int k = 0; k < 3; ++k) {
            lo3[k] = std::max(-x[k], -delta);
            hi3[k] = std::min(1.0 - x[k], delta);
        }
        if (qp3(B, g, a, c, lo3, hi3, d, &lq) != 0) raise(PA_ENUMERIC, "SQP subproblem has no solution");
        double dn = 0;
        for (int k = 0; k < 3; ++k) dn = std::max(dn, std::fabs(d[k]));
        if (dn < 1e-10) { r.converged = std::fabs(c) <= o.tol_c ? 2 : 0; break; }
        rho = std::max(rho, 2.0 * std::fabs(lq) + 1e-8);
        const double phi0 = f + rho * std::fabs(c);
        double gd = 0;
        for (int k = 0; k < 3; ++k) gd += g[k] * d[k];
        // directional derivative of the merit along d (the QP step removes the violation it can)
        double cd = c;
        for (int k = 0; k < 3; ++k) cd += a[k] * d[k];
        const double D = gd + rho * (std::fabs(cd) - std::fabs(c));
        double alpha = 1.0, xn[3], qn[2], dqn[6];
        bool acc = false;
        for (int t = 0; t < 6 && !acc; ++t, alpha *= 0.5) {
            for (int k = 0; k < 3; ++k) xn[k] = std::min(std::max(x[k] + alpha * d[k], 0.0), 1.0);
            to_mu(xn, m);
            if (!evaluate(m, false, qn, dqn)) continue;
            const double phi = fval(qn) + rho * std::fabs(cval(qn));
            if (phi <= phi0 + 1e-4 * alpha * std::min(D, 0.0) || (D >= 0 && phi < phi0)) acc = true;
            if (acc) break;
        }
        if (!acc) {
            delta *= 0.25;
            set_params(mu);   // back to the current point's parameters (its orbit is kept in uper)
            if (delta < 1e-6) break;
            ++r.iterations;
            record();
            continue;
        }
        // the accepted point's gradient (shoot again from its orbit: one more cheap period)
        get_state(0, uper.data(), nu);
        to_mu(xn, m);
        if (!evaluate(m, true, qn, dqn)) raise(PA_ENOCONV, "shooting failed at an accepted point");
        get_state(0, uper.data(), nu);
        double gn[3], an[3];
        for (int k = 0; k < 3; ++k) {
            gn[k] = o.obj_sign * dqn[3 * o.obj + k] * sc[k];
            an[k] = constrained ? dqn[3 * o.con + k] * sc[k] : 0.0;
        }
        // damped BFGS on the Hessian of the Lagrangian with the QP multiplier
        double sv[3], yv[3], Bs[3] = { 0, 0, 0 }, sBs = 0, sy = 0;
        for (int k = 0; k < 3; ++k) {
            sv[k] = xn[k] - x[k];
            yv[k] = (gn[k] - lq * an[k]) - (g[k] - lq * a[k]);
        }
        for (int k = 0; k < 3; ++k)
            for (int j = 0; j < 3; ++j) Bs[k] += B[k * 3 + j] * sv[j];
        for (int k = 0; k < 3; ++k) { sBs += sv[k] * Bs[k]; sy += sv[k] * yv[k]; }
        if (sBs > 0) {
            const double th = sy >= 0.2 * sBs ? 1.0 : 0.8 * sBs / (sBs - sy);
            double rv[3], sr = 0;
            for (int k = 0; k < 3; ++k) rv[k] = th * yv[k] + (1 - th) * Bs[k];
            for (int k = 0; k < 3; ++k) sr += sv[k] * rv[k];
            if (sr > 0)
                for (int k = 0; k < 3; ++k)
                    for (int j = 0; j < 3; ++j) B[k * 3 + j] += rv[k] * rv[j] / sr - Bs[k] * Bs[j] / sBs;
        }
        if (alpha >= 1.0 && dn >= 0.99 * delta) delta = std::min(2.0 * delta, 1.0);
        for (int k = 0; k < 3; ++k) { x[k] = xn[k]; g[k] = gn[k]; a[k] = an[k]; }
        q[0] = qn[0];
        q[1] = qn[1];
        f = fval(q);
        c = cval(q);
        lam = lq;
        to_mu(x, mu);
        ++r.iterations;
        record();
    }
    to_mu(x, mu);
    set_params(mu);
    set_state(uper.data(), nu);
    r.lam = lam;
    for (int k = 0; k < 3; ++k) r.mu[k] = mu[k];
    r.ms = now_ms() - t0;
    if (rep) *rep = r;
}

pa_status pa_optimize(pa_ctx* c, const pa_opt_opts* o, double mu[3], pa_opt_report* rep)
{
    return guard(c, [&] {
        if (!o || !mu) raise(PA_EINVAL, "NULL argument");
        if (o->obj < 0 || o->obj > 1 || o->con > 1 || (o->con >= 0 && o->con == o->obj) || o->maxit < 0 ||
            !(o->shoot_tol > 0) || !(o->shoot_eta > 0) || !(o->adj_rtol > 0) || o->shoot_maxit < 0)
            raise(PA_EINVAL, "bad optimisation options");
        c->optimize(*o, mu, rep);
    });
}
pa_status pa_dbg_qp3(const double B[9], const double g[3], const double a[3], double cval, const double lo[3],
                     const double hi[3], double d[3], double* lam)
{
    if (!B || !g || !a || !lo || !hi || !d || !lam) {
        g_create_err = "NULL argument";
        return PA_EINVAL;
    }
    if (qp3(B, g, a, cval, lo, hi, d, lam) != 0) {
        g_create_err = "no face of the box gives a solution";
        return PA_ENUMERIC;
    }
    return PA_OK;
}
// Prolongation of a state of a coarser O-grid discretisation to the nodes of
// `fine`: each fine node X (in the fixed reference domain) is located in the
// coarse triangle that contains it -- among the coarse quads around its
// polar cell, the triangle whose smallest barycentric coordinate is largest
// (a node between a coarse chord and the circle, where the coarse mesh does
// not reach, takes the nearest triangle's polynomial) -- and the coarse
// degree-p_c Lagrange interpolant of U_X is evaluated there.  Host only.
pa_status pa_prolong(const pa_config* coarse, const double* u_coarse, pa_ctx* fine, double* u_fine)
{
    if (!fine) return PA_EINVAL;
    return guard(fine, [&] {
        if (!coarse || !u_coarse || !u_fine) raise(PA_EINVAL, "NULL argument");
        const pa_config& C = *coarse;
        if (C.Nr < 1 || C.Nth < 3 || C.p < 1 || C.p > 3) raise(PA_EINVAL, "bad coarse discretisation");
        if (std::fabs(C.r_far - fine->cfg.r_far) > 1e-14 || std::fabs(C.stretch - fine->cfg.stretch) > 1e-14)
            raise(PA_EINVAL, "coarse and fine O-grids must share the far-field radius and stretching");
        const int Nr = C.Nr, Nth = C.Nth, pc = C.p, npc = (pc + 1) * (pc + 2) / 2;
        std::vector<double> rad(Nr + 1);
        const double q = std::pow(C.stretch, 8.0 / Nr), qN = std::pow(q, Nr);
        for (int i = 0; i <= Nr; ++i) rad[i] = 1.0 + (C.r_far - 1.0) * (std::pow(q, i) - 1.0) / (qN - 1.0);
        auto vert = [&](int i, int j, double* X) {
            const double th = 2.0 * M_PI * (((j % Nth) + Nth) % Nth) / Nth;
            X[0] = rad[i] * std::cos(th);
            X[1] = rad[i] * std::sin(th);
        };
        const Basis basis(pc);
        const int64_t nnf = (int64_t)fine->num_elems() * (fine->block_size() / 4);
        std::vector<double> xy(2 * nnf), phi(npc), dphi_buf(2 * npc);
        fine->node_coords(xy.data());
        for (int64_t k = 0; k < nnf; ++k) {
            const double X = xy[2 * k], Y = xy[2 * k + 1];
            const double r = std::sqrt(X * X + Y * Y);
            double th = std::atan2(Y, X);
            if (th < 0) th += 2.0 * M_PI;
            const int j0 = std::min((int)(th / (2.0 * M_PI / Nth)), Nth - 1);
            int i0 = 0;
            while (i0 + 1 < Nr && rad[i0 + 1] <= r) ++i0;
            double best = -1e300, bs = 0, bt = 0;
            int bestK = -1;
            for (int di = -1; di <= 1; ++di)
                for (int dj = -1; dj <= 1; ++dj) {
                    const int i = i0 + di, j = j0 + dj;
                    if (i < 0 || i >= Nr) continue;
                    double a[2], b[2], cc[2], d[2];
                    vert(i, j, a); vert(i + 1, j, b); vert(i + 1, j + 1, cc); vert(i, j + 1, d);
                    const double* tri[2][3] = { { a, b, cc }, { a, cc, d } };
                    for (int h = 0; h < 2; ++h) {
                        const double *p0 = tri[h][0], *p1 = tri[h][1], *p2 = tri[h][2];
                        const double j00 = p1[0] - p0[0], j01 = p2[0] - p0[0], j10 = p1[1] - p0[1], j11 = p2[1] - p0[1];
                        const double det = j00 * j11 - j01 * j10;
                        const double s_ = ((X - p0[0]) * j11 - (Y - p0[1]) * j01) / det;
                        const double t_ = (-(X - p0[0]) * j10 + (Y - p0[1]) * j00) / det;
                        const double mn = std::min({ s_, t_, 1.0 - s_ - t_ });
                        if (mn > best) {
                            best = mn; bs = s_; bt = t_;
                            bestK = 2 * (i * Nth + (((j % Nth) + Nth) % Nth)) + h;
                        }
                    }
                }
            basis.eval(bs, bt, phi.data(), reinterpret_cast<double(*)[2]>(dphi_buf.data()));
            for (int m = 0; m < 4; ++m) {
                double v = 0.0;
                for (int a = 0; a < npc; ++a) v += phi[a] * u_coarse[((int64_t)bestK * npc + a) * 4 + m];
                u_fine[4 * k + m] = v;
            }
        }
    });
}
pa_status pa_ws_pod(pa_ctx* c, int32_t kmax, double* mean, double* modes, double* eig, int32_t* k)
{
    return guard(c, [&] {
        if (kmax < 0) raise(PA_EINVAL, "kmax must be non-negative");
        const int n = c->ws_pod(kmax, mean, modes, eig);
        if (k) *k = n;
    });
}
pa_status pa_ws_save(pa_ctx* c, const char* path)
{
    return guard(c, [&] {
        if (!path) raise(PA_EINVAL, "no path");
        c->ws_save(path);
    });
}
pa_status pa_ws_load(pa_ctx* c, const char* path)
{
    return guard(c, [&] {
        if (!path) raise(PA_EINVAL, "no path");
        c->ws_load(path);
    });
}

// ---- allocation-free perceptron pass ----
// Work memory of pa_mlp_grad_noalloc: a file-scope device array of
// PA_MLP_SCRATCH_FLOATS floats (one copy per GPU, held until the process
// ends).  Host code never passes the array's name to a kernel (on the host
// it only stands in for the symbol): its device address is looked up once
// per device with hipGetSymbolAddress and that pointer is used.
static __device__ __align__(256) float scratch[PA_MLP_SCRATCH_FLOATS];
static std::mutex g_scratch_mu;
static float* g_scratch_ptr[64] = {};

static float* scratch_on_current_device()
{
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) raise(PA_EDEVICE, "device ordinal %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            raise(PA_EDEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<float*>(ptr);
    }
    return g_scratch_ptr[dev];
}

pa_status pa_mlp_grad_noalloc(int32_t in, int32_t width, int32_t out, int32_t batch, const float* params,
                              const float* X, const float* T, float* loss, float* grads, void* stream)
{
    if (in < 1 || width < 1 || out < 1 || batch < 1 || !params || !X || !T || !loss || !grads) {
        g_create_err = "bad arguments";
        return PA_EINVAL;
    }
    try {
        const MlpShape sh(in, width, out);
        // activations H_1..H_4 and the two back-propagation buffers
        const int64_t need = ((int64_t)3 * width + out + 2 * (int64_t)sh.maxw) * batch;
        if (need > PA_MLP_SCRATCH_FLOATS) {
            g_create_err = "perceptron pass needs " + std::to_string(need) + " floats of work memory, more than the " +
                           std::to_string((long long)PA_MLP_SCRATCH_FLOATS) + " available";
            return PA_EINVAL;
        }
        float* w = scratch_on_current_device();
        float* H[4];
        for (int l = 0; l < 4; ++l) {
            H[l] = w;
            w += (int64_t)sh.dims[l + 1] * batch;
        }
        float* dA = w;
        float* dB = dA + (int64_t)sh.maxw * batch;
        hipStream_t st = static_cast<hipStream_t>(stream);
        mlp_forward(sh, params, X, H, batch, st);
        mlp_mse(sh, H, T, dA, batch, loss, st);
        mlp_backward(sh, params, X, H, dA, dB, grads, batch, st);
        return PA_OK;
    } catch (const PaError& e) {
        g_create_err = e.msg;
        return e.code;
    }
}

pa_status pa_dbg_mlp(int32_t in, int32_t width, int32_t out, int32_t batch, const float* params, const float* X,
                     const float* T, float* loss, float* grads)
{
    if (in < 1 || width < 1 || out < 1 || batch < 1 || !params || !X || !T || !loss || !grads) {
        g_create_err = "bad arguments";
        return PA_EINVAL;
    }
    hipStream_t st = nullptr;
    try {
        HIPCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        {
            Mlp m;
            m.init(in, width, out, st);
            m.reserve(batch);
            HIPCHK(hipMemcpyAsync(m.p, params, sizeof(float) * m.nparam, hipMemcpyHostToDevice, st));
            HIPCHK(hipMemcpyAsync(m.X, X, sizeof(float) * (size_t)in * batch, hipMemcpyHostToDevice, st));
            HIPCHK(hipMemcpyAsync(m.T, T, sizeof(float) * (size_t)out * batch, hipMemcpyHostToDevice, st));
            m.forward(batch);
            m.mse(batch);
            m.backward(batch);
            HIPCHK(hipMemcpyAsync(loss, m.loss, sizeof(float), hipMemcpyDeviceToHost, st));
            HIPCHK(hipMemcpyAsync(grads, m.g, sizeof(float) * m.nparam, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
        }
        (void)hipStreamDestroy(st);
        return PA_OK;
    } catch (const PaError& e) {
        if (st) (void)hipStreamDestroy(st);
        g_create_err = e.msg;
        return e.code;
    }
}

pa_status pa_batch_gradients(const pa_config* cfg, int32_t n, const double* mu, const pa_batch_opts* o,
                             double* qoi, double* dJ, double* per, double* states, double* dJd)
{
    if (!cfg || !mu || !o || n < 0 || o->workers < 1 || o->shoot_maxit < 0) {
        g_create_err = "bad batch arguments";
        return PA_EINVAL;
    }
    std::atomic<int> next{ 0 };
    std::mutex mtx;
    pa_status first = PA_OK;
    std::string first_msg;
    auto fail = [&](pa_status rc, const std::string& msg) {
        std::lock_guard<std::mutex> lk(mtx);
        if (first == PA_OK) { first = rc; first_msg = msg; }
        next.store(n);   // stop handing out instances
    };
    auto worker = [&]() {
        pa_ctx* c = nullptr;
        pa_status rc = pa_create(cfg, &c);
        if (rc != PA_OK) { fail(rc, pa_last_error(nullptr)); return; }
        for (;;) {
            const int i = next.fetch_add(1);
            if (i >= n) break;
            double q[2], g[6], res = 0.0;
            rc = pa_set_params(c, mu + 3 * (int64_t)i);
            if (rc == PA_OK) rc = pa_set_freestream(c, nullptr);
            if (rc == PA_OK) {
                if (o->shoot_maxit > 0) {
                    pa_shoot_report rep{};
                    rc = pa_shoot(c, o->shoot_tol, o->shoot_eta, o->shoot_maxit, &rep);
                    if (rc == PA_ENOCONV && o->allow_unconverged && rep.newton_its >= o->shoot_maxit) rc = PA_OK;
                    res = rep.res;
                } else {
                    double qq[2];
                    rc = pa_primal_period(c, qq, &res);
                }
            }
            if (rc == PA_OK && states)
                rc = pa_get_state(c, 0, states + (int64_t)i * pa_num_dofs(c), pa_num_dofs(c));
            if (rc == PA_OK) rc = pa_adjoint_gradient(c, o->adj_rtol, q, g, nullptr);
            double gd[6];
            if (rc == PA_OK && dJd) rc = pa_tangent_gradient(c, o->adj_rtol, gd, nullptr);
            if (rc != PA_OK && o->keep_going && rc != PA_EDEVICE && rc != PA_ENOMEM) {
                const double nan = std::nan("");
                if (qoi) qoi[2 * (int64_t)i] = qoi[2 * (int64_t)i + 1] = nan;
                if (dJ) for (int k = 0; k < 6; ++k) dJ[6 * (int64_t)i + k] = nan;
                if (dJd) for (int k = 0; k < 6; ++k) dJd[6 * (int64_t)i + k] = nan;
                if (per) per[i] = nan;
                continue;
            }
            if (rc != PA_OK) {
                fail(rc, std::string("instance ") + std::to_string(i) + ": " + pa_last_error(c));
                break;
            }
            if (qoi) { qoi[2 * (int64_t)i] = q[0]; qoi[2 * (int64_t)i + 1] = q[1]; }
            if (dJ) for (int k = 0; k < 6; ++k) dJ[6 * (int64_t)i + k] = g[k];
            if (dJd) for (int k = 0; k < 6; ++k) dJd[6 * (int64_t)i + k] = gd[k];
            if (per) per[i] = res;
        }
        pa_destroy(c);
    };
    std::vector<std::thread> pool;
    const int nw = std::min<int>(o->workers, std::max(n, 1));
    for (int w = 0; w < nw; ++w) pool.emplace_back(worker);
    for (auto& t : pool) t.join();
    if (first != PA_OK) g_create_err = first_msg;
    return first;
}

pa_status pa_shoot(pa_ctx* c, double tol, double eta, int32_t maxit, pa_shoot_report* rep)
{
    return guard(c, [&] {
        if (!(tol > 0) || !(eta > 0) || maxit < 0) raise(PA_EINVAL, "bad shooting options");
        c->shoot(tol, eta, maxit, rep);
    });
}
pa_status pa_shoot_descent(pa_ctx* c, double tol, int32_t memory, int32_t maxit, pa_shoot_report* rep)
{
    return guard(c, [&] {
        if (!(tol > 0) || memory < 0 || memory > 32 || maxit < 0) raise(PA_EINVAL, "bad descent options");
        c->shoot_descent(tol, memory, maxit, rep);
    });
}
pa_status pa_periodicity_gradient(pa_ctx* c, double* grad, double* j)
{
    return guard(c, [&] {
        const double v = c->periodicity_gradient(grad);
        if (j) *j = v;
    });
}
pa_status pa_floquet(pa_ctx* c, int32_t k, uint64_t seed, double* re, double* im, int32_t* nritz, double* hsub)
{
    return guard(c, [&] {
        if (!re || !im) raise(PA_EINVAL, "no output");
        const int n = c->floquet(k, seed, re, im, hsub);
        if (nritz) *nritz = n;
    });
}
pa_status pa_fixed_point(pa_ctx* c, int32_t periods, double* res)
{
    return guard(c, [&] {
        if (periods < 0) raise(PA_EINVAL, "negative period count");
        c->fixed_point(periods, res);
    });
}
pa_status pa_adjoint_gradient(pa_ctx* c, double rtol, double qoi[2], double dJ[6], pa_adjoint_report* rep)
{
    return guard(c, [&] {
        if (!dJ || !(rtol > 0)) raise(PA_EINVAL, "bad arguments");
        c->adjoint_gradient(rtol, qoi, dJ, rep);
    });
}
pa_status pa_tangent_gradient(pa_ctx* c, double rtol, double dJ[6], int32_t its[3])
{
    return guard(c, [&] {
        if (!dJ || !(rtol > 0.0)) raise(PA_EINVAL, "bad arguments");
        c->tangent_gradient(rtol, dJ, its);
    });
}

pa_status pa_tangent_sweep(pa_ctx* c, const double* v, double* out)
{
    return guard(c, [&] { if (!v || !out) raise(PA_EINVAL, "null vector"); c->tangent_sweep_h(v, out); });
}
pa_status pa_adjoint_sweep(pa_ctx* c, const double* lam, int32_t fq, double* lam0, double* grad)
{
    return guard(c, [&] {
        if (!lam || !lam0 || fq > 1 || (fq >= 0 && !grad)) raise(PA_EINVAL, "bad arguments");
        c->adjoint_sweep_h(lam, fq, lam0, grad);
    });
}
pa_status pa_dbg_gbar(pa_ctx* c, int32_t n, int32_t i, double* out)
{
    return guard(c, [&] { c->dbg_gbar(n, i, out, false); });
}
pa_status pa_dbg_dgbar(pa_ctx* c, int32_t n, int32_t i, double* out)
{
    return guard(c, [&] { c->dbg_gbar(n, i, out, true); });
}
pa_status pa_dbg_residual(pa_ctx* c, int32_t n, int32_t i, const double* u, double* r)
{
    return guard(c, [&] { c->dbg_residual(n, i, u, r, false); });
}
pa_status pa_dbg_jacobian(pa_ctx* c, int32_t n, int32_t i, const double* u, double* blk)
{
    return guard(c, [&] { c->dbg_jacobian(n, i, u, blk); });
}
pa_status pa_dbg_dr_dmu(pa_ctx* c, int32_t n, int32_t i, const double* u, double* out)
{
    return guard(c, [&] { c->dbg_residual(n, i, u, out, true); });
}
pa_status pa_dbg_qoi(pa_ctx* c, int32_t n, int32_t i, const double* u, double f[2], double* dfdu, double* dfdmu)
{
    return guard(c, [&] { c->dbg_qoi(n, i, u, f, dfdu, dfdmu); });
}
pa_status pa_dbg_bsr_apply(pa_ctx* c, const double* blk, double alpha, double beta, int32_t tr, const double* x,
                           double* y)
{
    return guard(c, [&] { c->dbg_bsr_apply(blk, alpha, beta, tr, x, y); });
}
pa_status pa_dbg_blockinv(pa_ctx* c, const double* blk, double adt, double* out)
{
    return guard(c, [&] { c->dbg_blockinv(blk, adt, out); });
}
pa_status pa_dbg_stage_solve(pa_ctx* c, const double* blk, double adt, int32_t tr, const double* rhs, double* x,
                             int32_t* iters)
{
    return guard(c, [&] {
        int its = c->dbg_stage_solve(blk, adt, tr, rhs, x);
        if (iters) *iters = its;
    });
}
pa_status pa_dbg_traj(pa_ctx* c, int32_t which, int32_t n, int32_t i, double* out)
{
    return guard(c, [&] { c->dbg_traj(which, n, i, out); });
}
pa_status pa_set_timing(pa_ctx* c, int32_t on) { return guard(c, [&] { c->set_timing(on != 0); }); }
pa_status pa_kernel_time(pa_ctx* c, int32_t k, double* ms, int64_t* cnt)
{
    return guard(c, [&] { c->kernel_time(k, ms, cnt); });
}
pa_status pa_kernel_skipped(pa_ctx* c, int32_t k, int64_t* skipped)
{
    return guard(c, [&] {
        if (!skipped) raise(PA_EINVAL, "null output");
        *skipped = c->kernel_skipped(k);
    });
}
pa_status pa_kernel_vectors(pa_ctx* c, int32_t k, int64_t* vectors)
{
    return guard(c, [&] {
        if (!vectors) raise(PA_EINVAL, "null output");
        *vectors = c->kernel_vectors(k);
    });
}
pa_status pa_bench_copy(pa_ctx* c, int32_t reps, double* avg, int64_t* bytes)
{
    return guard(c, [&] {
        if (reps < 1 || !avg) raise(PA_EINVAL, "bad arguments");
        *avg = c->bench_copy(reps, bytes);
    });
}
pa_status pa_tuning(pa_ctx* c, int32_t* fwd_chunks, double fwd_us[3])
{
    return guard(c, [&] { c->tuning(fwd_chunks, fwd_us); });
}

pa_status pa_bench_spmv_lo(pa_ctx* c, int32_t reps, int32_t tr, double* avg)
{
    return guard(c, [&] {
        if (!avg || reps < 1) raise(PA_EINVAL, "bad arguments");
        *avg = c->bench_spmv_lo(reps, tr);
    });
}

pa_status pa_bench_spmv_m(pa_ctx* c, int32_t reps, int32_t tr, int32_t nrhs, double* avg)
{
    if (!avg) return c ? (c->err = "NULL output", PA_EINVAL) : PA_EINVAL;
    return guard(c, [&] { *avg = c->bench_spmv_m(reps, tr, nrhs); });
}
pa_status pa_bench_spmv(pa_ctx* c, int32_t reps, int32_t tr, double* avg)
{
    return guard(c, [&] {
        if (reps < 1 || !avg) raise(PA_EINVAL, "bad arguments");
        *avg = c->bench_spmv(reps, tr);
    });
}

}  // extern "C"
