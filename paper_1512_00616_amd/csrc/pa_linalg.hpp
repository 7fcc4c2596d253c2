// Block-sparse and Krylov kernels of the periodic-adjoint library (gfx950).
//
// Operators of one DIRK stage (arXiv:1512.00616 Sec. 2.2 eq. dirk):
//   A_i = M - dt a_ii dr/du(u_i),  M = blockdiag(2|K| Mhat (x) I_4)  (constant)
// dr/du is stored as fixed-width block rows: row K holds its diagonal block
// and the blocks coupling K to its neighbours across faces 0, 1, 2.
//
// * k_bsr_apply:   y = alpha M x + beta J x   or   y = alpha M x + beta J^T x.
//   One wave per block row; every block is streamed from HBM with coalesced
//   16-byte loads into LDS (each byte read once) and reduced from there.
//   J^T is a gather: row K of J^T takes the diagonal block transposed and,
//   for each neighbour, the neighbour's block that points back at K (its
//   slot 1 + twin) transposed -- no atomics.
// * k_blockinv:    block-Jacobi preconditioner: LU with partial pivoting of
//   every diagonal block of A_i in LDS, then the explicit inverse.
// * GMRES vector kernels with fixed-order (deterministic) reductions.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pa {

// y = alpha * M x + beta * op(J) x
template <int NP>
__global__ void __launch_bounds__(64) k_bsr_apply(int Ne, const int32_t* __restrict__ enb,
                                                  const int8_t* __restrict__ etw, const double* __restrict__ area,
                                                  const double* __restrict__ mh, const double* __restrict__ J,
                                                  const double* __restrict__ x, double* __restrict__ y,
                                                  double alpha, double beta, int trans)
{
    constexpr int B = 4 * NP, BB = B * B;
    __shared__ double sblk[B][B + 1];
    __shared__ double sx[B];
    const int K = blockIdx.x, lane = threadIdx.x;
    double acc = 0.0;
    for (int s = 0; s < 4; ++s) {
        int src, xe;
        if (s == 0) { src = K * 4; xe = K; }
        else {
            int nb = enb[3 * K + s - 1];
            if (nb < 0) continue;
            xe = nb;
            src = trans ? nb * 4 + 1 + etw[3 * K + s - 1] : K * 4 + s;
        }
        if (beta == 0.0) continue;
        const double2* blk2 = reinterpret_cast<const double2*>(J + (int64_t)src * BB);
        for (int t = lane; t < BB / 2; t += 64) {
            double2 v = blk2[t];
            int e = 2 * t;
            sblk[e / B][e % B] = v.x;
            sblk[(e + 1) / B][(e + 1) % B] = v.y;
        }
        if (lane < B) sx[lane] = x[(int64_t)xe * B + lane];
        __syncthreads();
        if (lane < B) {
            double a = 0.0;
            if (!trans) {
#pragma unroll 8
                for (int j = 0; j < B; ++j) a += sblk[lane][j] * sx[j];
            } else {
#pragma unroll 8
                for (int i = 0; i < B; ++i) a += sblk[i][lane] * sx[i];
            }
            acc += a;
        }
        __syncthreads();
    }
    if (lane < B) {
        int a = lane >> 2, m = lane & 3;
        double mv = 0.0;
        if (alpha != 0.0) {
            const double* xK = x + (int64_t)K * B;
            for (int b = 0; b < NP; ++b) mv += mh[a * NP + b] * xK[b * 4 + m];
            mv *= 2.0 * area[K];
        }
        y[(int64_t)K * B + lane] = alpha * mv + beta * acc;
    }
}

// inverse of every diagonal block of A = M - c J (partial pivoting, lowest
// row on ties); Ainv [Ne][B][B] row-major
template <int NP>
__global__ void __launch_bounds__(64) k_blockinv(int Ne, const double* __restrict__ area, const double* __restrict__ mh,
                                                 const double* __restrict__ J, double c, double* __restrict__ Ainv,
                                                 int* __restrict__ status)
{
    constexpr int B = 4 * NP, BB = B * B;
    __shared__ double a[B][B + 1];
    __shared__ double inv[B][B + 1];
    __shared__ int piv[B];
    __shared__ int sp;
    const int K = blockIdx.x, lane = threadIdx.x;
    const double* src = J + (int64_t)K * 4 * BB;
    const double s2 = 2.0 * area[K];
    for (int t = lane; t < BB; t += 64) {
        int i = t / B, j = t % B;
        double mm = ((i & 3) == (j & 3)) ? s2 * mh[(i >> 2) * NP + (j >> 2)] : 0.0;
        a[i][j] = mm - c * src[t];
    }
    __syncthreads();
    for (int k = 0; k < B; ++k) {
        if (lane == 0) {
            int p = k;
            double best = fabs(a[k][k]);
            for (int i = k + 1; i < B; ++i) {
                double v = fabs(a[i][k]);
                if (v > best) { best = v; p = i; }
            }
            piv[k] = p;
            sp = p;
            if (best == 0.0) status[0] = 1;
        }
        __syncthreads();
        int p = sp;
        if (p != k) {
            for (int j = lane; j < B; j += 64) {
                double t = a[k][j];
                a[k][j] = a[p][j];
                a[p][j] = t;
            }
        }
        __syncthreads();
        double d = a[k][k];
        for (int i = k + 1 + lane; i < B; i += 64) a[i][k] /= d;
        __syncthreads();
        for (int t = lane; t < (B - k - 1) * (B - k - 1); t += 64) {
            int i = k + 1 + t / (B - k - 1), j = k + 1 + t % (B - k - 1);
            a[i][j] -= a[i][k] * a[k][j];
        }
        __syncthreads();
    }
    // column c of the inverse solves L U x = P e_c (each lane owns one column of inv)
    if (lane < B) {
        const int col = lane;
        for (int i = 0; i < B; ++i) inv[i][col] = (i == col) ? 1.0 : 0.0;
        for (int k = 0; k < B; ++k) {
            int p = piv[k];
            if (p != k) { double t = inv[k][col]; inv[k][col] = inv[p][col]; inv[p][col] = t; }
        }
        for (int i = 0; i < B; ++i) {
            double s = inv[i][col];
            for (int j = 0; j < i; ++j) s -= a[i][j] * inv[j][col];
            inv[i][col] = s;
        }
        for (int i = B - 1; i >= 0; --i) {
            double s = inv[i][col];
            for (int j = i + 1; j < B; ++j) s -= a[i][j] * inv[j][col];
            inv[i][col] = s / a[i][i];
        }
    }
    __syncthreads();
    double* dst = Ainv + (int64_t)K * BB;
    for (int t = lane; t < BB; t += 64) dst[t] = inv[t / B][t % B];
}

// z_K = Ainv_K x_K  (trans: Ainv_K^T x_K)
template <int NP>
__global__ void __launch_bounds__(64) k_block_apply(int Ne, const double* __restrict__ Ainv,
                                                    const double* __restrict__ x, double* __restrict__ z, int trans)
{
    constexpr int B = 4 * NP, BB = B * B;
    __shared__ double sblk[B][B + 1];
    __shared__ double sx[B];
    const int K = blockIdx.x, lane = threadIdx.x;
    const double2* blk2 = reinterpret_cast<const double2*>(Ainv + (int64_t)K * BB);
    for (int t = lane; t < BB / 2; t += 64) {
        double2 v = blk2[t];
        int e = 2 * t;
        sblk[e / B][e % B] = v.x;
        sblk[(e + 1) / B][(e + 1) % B] = v.y;
    }
    if (lane < B) sx[lane] = x[(int64_t)K * B + lane];
    __syncthreads();
    if (lane < B) {
        double a = 0.0;
        if (!trans)
            for (int j = 0; j < B; ++j) a += sblk[lane][j] * sx[j];
        else
            for (int i = 0; i < B; ++i) a += sblk[i][lane] * sx[i];
        z[(int64_t)K * B + lane] = a;
    }
}

// ------------------------------------------------------------------ vector kernels
constexpr int RED_THREADS = 256;
constexpr int RED_BLOCKS = 512;

// partial[blk][c] = sum over the block's chunk of w . V_c, c < ncols (V_c = V + c*ldv)
__global__ void __launch_bounds__(RED_THREADS) k_multidot(const double* __restrict__ V, int64_t ldv, int ncols,
                                                          const double* __restrict__ w, int64_t n,
                                                          double* __restrict__ partial)
{
    __shared__ double red[RED_THREADS];
    const int tid = threadIdx.x;
    int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    int64_t lo = blockIdx.x * chunk, hi = lo + chunk < n ? lo + chunk : n;
    for (int c = 0; c < ncols; ++c) {
        const double* v = V + (int64_t)c * ldv;
        double s = 0.0;
        for (int64_t i = lo + tid; i < hi; i += RED_THREADS) s += w[i] * v[i];
        red[tid] = s;
        __syncthreads();
        for (int st = RED_THREADS / 2; st > 0; st >>= 1) {
            if (tid < st) red[tid] += red[tid + st];
            __syncthreads();
        }
        if (tid == 0) partial[(int64_t)blockIdx.x * ncols + c] = red[0];
        __syncthreads();
    }
}

// out[c] = sum_blk partial[blk][c] (fixed order)
__global__ void k_reduce_partials(const double* __restrict__ partial, int nblk, int ncols, double* __restrict__ out)
{
    int c = threadIdx.x;
    if (c >= ncols) return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += partial[(int64_t)b * ncols + c];
    out[c] = s;
}

// w += sign * sum_c h[c] V_c
__global__ void k_vupdate(const double* __restrict__ V, int64_t ldv, int ncols, const double* __restrict__ h,
                          double sign, double* __restrict__ w, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int c = 0; c < ncols; ++c) s += h[c] * V[(int64_t)c * ldv + i];
    w[i] += sign * s;
}

// y = a x + b y
__global__ void k_axpby(double a, const double* __restrict__ x, double b, double* __restrict__ y, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = a * x[i] + (b == 0.0 ? 0.0 : b * y[i]);
}

// z = a x + b y (out of place)
__global__ void k_lincomb(double a, const double* __restrict__ x, double b, const double* __restrict__ y,
                          double* __restrict__ z, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) z[i] = a * x[i] + b * y[i];
}

// stage Newton residual R = M k - dt r (M applied block-wise)
template <int NP>
__global__ void k_stage_residual(int Ne, const double* __restrict__ area, const double* __restrict__ mh,
                                 const double* __restrict__ k, const double* __restrict__ r, double dt,
                                 double* __restrict__ R)
{
    constexpr int B = 4 * NP;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)Ne * B) return;
    int K = (int)(i / B), l = (int)(i % B), a = l >> 2, m = l & 3;
    const double* kK = k + (int64_t)K * B;
    double s = 0.0;
    for (int b = 0; b < NP; ++b) s += mh[a * NP + b] * kK[b * 4 + m];
    R[i] = 2.0 * area[K] * s - dt * r[i];
}

}  // namespace pa
