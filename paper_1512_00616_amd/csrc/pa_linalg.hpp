// Block-sparse and Krylov kernels of the periodic-adjoint library (gfx950).
//
// Operators of one DIRK stage (arXiv:1512.00616 Sec. 2.1 eq. dirk):
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
// * k_blockprep / k_form_ahat / k_ahat_fwd / k_ahat_tr (below): the
//   block-Jacobi factor folded into the stored operator and its forward and
//   transposed applies (FP64, or FP32/BF16 copies for mixed precision).
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
                                                  double alpha, double beta, int trans, const int* __restrict__ skip)
{
    constexpr int B = 4 * NP, BB = B * B;
    __shared__ double sblk[B][B + 1];
    __shared__ double sx[B];
    if (skip && *skip) return;
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

// z_K = Ainv_K x_K  (trans: Ainv_K^T x_K)
template <int NP>
__global__ void __launch_bounds__(64) k_block_apply(int Ne, const double* __restrict__ Ainv,
                                                    const double* __restrict__ x, double* __restrict__ z, int trans,
                                                    const int* __restrict__ skip)
{
    constexpr int B = 4 * NP, BB = B * B;
    __shared__ double sblk[B][B + 1];
    __shared__ double sx[B];
    if (skip && *skip) return;
    const int K = blockIdx.x, lane = threadIdx.x;
    const double2* blk2 = reinterpret_cast<const double2*>(Ainv + (int64_t)K * BB);
    // every load issued before the first LDS store
    constexpr int H2 = BB / 2, NL = (H2 + 63) / 64;
    double2 v[NL];
#pragma unroll
    for (int u = 0; u < NL; ++u) v[u] = blk2[lane + 64 * u < H2 ? lane + 64 * u : H2 - 1];
    const double xv = x[(int64_t)K * B + (lane < B ? lane : 0)];
#pragma unroll
    for (int u = 0; u < NL; ++u) {
        const int t = lane + 64 * u;
        if (t < H2) {
            const int e = 2 * t;
            sblk[e / B][e % B] = v[u].x;
            sblk[(e + 1) / B][(e + 1) % B] = v[u].y;
        }
    }
    if (lane < B) sx[lane] = xv;
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

// Arnoldi state of one restart cycle kept in device memory so that the
// iterations run without host round trips.  Every iteration kernel returns
// at once when `done` is set; the host polls `done` every few iterations.
constexpr int GM_MAXM = 64;
struct GmState {
    double H[(GM_MAXM + 1) * GM_MAXM];   // Hessenberg (rotated), row-major (m+1) x m
    double cs[GM_MAXM], sn[GM_MAXM];
    double g[GM_MAXM + 1];
    double y[GM_MAXM];
    double hc[GM_MAXM + 2];              // Gram-Schmidt coefficients of the current column
    double tol;                          // absolute residual target
    double res;                          // current residual estimate
    int done;                            // 1: converged or happy breakdown
    int its;                             // columns of the cycle when done
};

// ------------------------------------------------------------------ vector kernels
// Multi-column dot products  s_c = <X_c, w>,  X_c = V + c*ldv (c < ncols),
// optionally followed by <w, w>, in one launch and in a fixed summation
// order (bitwise reproducible, no floating-point atomics):
//   1. block b covers MD_TILE consecutive entries; each thread holds two
//      double2 of w and, eight columns at a time, issues all sixteen
//      16-byte loads of those columns before using any of them;
//   2. the 32 per-thread products of a column group are summed over the
//      wave by a halving exchange (32 shuffles for 32 columns instead of
//      6 per column), then over the four waves through LDS;
//   3. the block's row of partials goes to `partial[b][nc]`; every block of
//      the next kernel sums the rows in the same fixed order (a
//      completion count inside one launch would need device-scope fences
//      in every block, which write back the XCD's L2 on this GPU).
constexpr int MD_THREADS = 256;
constexpr int MD_TILE = 4 * MD_THREADS;   // doubles per block
constexpr int MD_GROUP = 32;              // columns per reduction group
constexpr int MD_MAXC = 256;              // column limit of a launch
inline int64_t mdot_blocks(int64_t n) { return (n + MD_TILE - 1) / MD_TILE; }

// two consecutive entries (16- or 8-byte aligned) widened to double
__device__ __forceinline__ double2 ld2(const double* p) { return *reinterpret_cast<const double2*>(p); }
__device__ __forceinline__ double2 ld2(const float* p)
{
    const float2 f = *reinterpret_cast<const float2*>(p);
    return make_double2(f.x, f.y);
}
__device__ __forceinline__ void st2(double* p, double2 v) { *reinterpret_cast<double2*>(p) = v; }
__device__ __forceinline__ void st2(float* p, double2 v)
{
    *reinterpret_cast<float2*>(p) = make_float2((float)v.x, (float)v.y);
}

// Column sums over a wave: on entry every lane holds p[0..31]; on exit p[0]
// of lane l holds the wave total of column l >> 1.  Each halving exchange
// (offset o = 2K, K columns kept) sends the half of the columns the partner
// keeps; the lane with bit o set keeps the upper half.
template <int K>
__device__ __forceinline__ void colsum_halve(double (&p)[MD_GROUP], int lane)
{
    constexpr int o = 2 * K;
    const bool up = (lane & o) != 0;
#pragma unroll
    for (int c = 0; c < K; ++c) {
        const double keep = up ? p[c + K] : p[c];
        const double send = up ? p[c] : p[c + K];
        p[c] = keep + __shfl_xor(send, o, 64);
    }
    if constexpr (K > 1) colsum_halve<K / 2>(p, lane);
}
__device__ __forceinline__ void wave_colsum32(double (&p)[MD_GROUP])
{
    const int lane = threadIdx.x & 63;
    colsum_halve<MD_GROUP / 2>(p, lane);
    p[0] += __shfl_xor(p[0], 1, 64);
}

// Block total of the wave column sums: result for column u is valid in
// thread u (u < 32) after the call.
__device__ __forceinline__ double block_colsum32(double (&p)[MD_GROUP], double (*sred)[MD_GROUP])
{
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    wave_colsum32(p);
    if ((lane & 1) == 0) sred[wv][lane >> 1] = p[0];
    __syncthreads();
    double s = 0.0;
    if (tid < MD_GROUP)
#pragma unroll
        for (int k = 0; k < MD_THREADS / 64; ++k) s += sred[k][tid];
    __syncthreads();
    return s;
}

// Phase 1: this block's partial sums, written to partial[blockIdx.x][nc]
// with nc = ncols + with_ww.  Requires n even and 16-byte aligned columns.
template <class T>
__device__ __forceinline__ void mdot_partials(const T* __restrict__ V, int64_t ldv, int ncols, int with_ww,
                                              const T* __restrict__ w, int64_t n, double* __restrict__ partial)
{
    __shared__ double sred[MD_THREADS / 64][MD_GROUP];
    const int tid = threadIdx.x;
    const int nc = ncols + with_ww;
    const int64_t i0 = (int64_t)blockIdx.x * MD_TILE + 2 * tid, i1 = i0 + 2 * MD_THREADS;
    const bool in0 = i0 < n, in1 = i1 < n;
    const int64_t a0 = in0 ? i0 : 0, a1 = in1 ? i1 : 0;   // clamped (valid) addresses
    double2 w0 = make_double2(0.0, 0.0), w1 = make_double2(0.0, 0.0);
    if (in0) w0 = ld2(w + i0);
    if (in1) w1 = ld2(w + i1);
    const double ww = w0.x * w0.x + w0.y * w0.y + w1.x * w1.x + w1.y * w1.y;
    for (int g0 = 0; g0 < nc; g0 += MD_GROUP) {
        double p[MD_GROUP];
#pragma unroll
        for (int q = 0; q < MD_GROUP / 8; ++q) {
            const int cb = g0 + 8 * q;
            if (cb < nc) {
                double2 a[8], b[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int c = cb + u;
                    const T* vc = V + (int64_t)(c < ncols ? c : ncols - 1) * ldv;
                    a[u] = ld2(vc + a0);
                    b[u] = ld2(vc + a1);
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int c = cb + u;
                    const double s = a[u].x * w0.x + a[u].y * w0.y + b[u].x * w1.x + b[u].y * w1.y;
                    p[8 * q + u] = c < ncols ? s : (c == ncols && with_ww ? ww : 0.0);
                }
            } else {
#pragma unroll
                for (int u = 0; u < 8; ++u) p[8 * q + u] = 0.0;
            }
        }
        const double s = block_colsum32(p, sred);
        if (tid < MD_GROUP && g0 + tid < nc) partial[(int64_t)blockIdx.x * nc + g0 + tid] = s;
    }
}

// Phase 2: out[c] = sum over blocks (block order within each thread's row
// set, then the fixed exchange tree) of partial[b][c], c < nc; out in LDS.
// Every block that calls it gets the same bits.
__device__ __forceinline__ void mdot_finish(const double* __restrict__ partial, int nblk, int nc, double* out)
{
    __shared__ double sred[MD_THREADS / 64][MD_GROUP];
    const int tid = threadIdx.x;
    for (int g0 = 0; g0 < nc; g0 += MD_GROUP) {
        double p[MD_GROUP];
#pragma unroll
        for (int u = 0; u < MD_GROUP; ++u) p[u] = 0.0;
        for (int b = tid; b < nblk; b += MD_THREADS) {
            const double* row = partial + (int64_t)b * nc;
            double v[MD_GROUP];
#pragma unroll
            for (int u = 0; u < MD_GROUP; ++u) v[u] = row[g0 + u < nc ? g0 + u : nc - 1];
#pragma unroll
            for (int u = 0; u < MD_GROUP; ++u) p[u] += g0 + u < nc ? v[u] : 0.0;
        }
        const double s = block_colsum32(p, sred);
        if (tid < MD_GROUP && g0 + tid < nc) out[g0 + tid] = s;
    }
    __syncthreads();
}

// Eight-column variant of the wave sums: on exit p[0] of lane l holds the
// wave total of column (l >> 3) & 7 for lanes with l % 8 == 0 (halving
// exchanges at offsets 32, 16, 8, then plain sums over the low three bits).
__device__ __forceinline__ void wave_colsum8(double (&p)[8])
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        const int k = 4 >> s, o = 32 >> s;
        const bool up = (lane & o) != 0;
#pragma unroll
        for (int c = 0; c < k; ++c) {
            const double keep = up ? p[c + k] : p[c];
            const double send = up ? p[c] : p[c + k];
            p[c] = keep + __shfl_xor(send, o, 64);
        }
    }
    p[0] += __shfl_xor(p[0], 4, 64);
    p[0] += __shfl_xor(p[0], 2, 64);
    p[0] += __shfl_xor(p[0], 1, 64);
}

// One block's partial sums of eight columns cb..cb+7 (those < nc = ncols +
// with_ww; column ncols is <w, w> when with_ww) over its MD_TILE entries,
// written to partial[blockIdx.x][nc].
template <class T>
__device__ __forceinline__ void mdot_chunk8(const T* __restrict__ V, int64_t ldv, int ncols, int with_ww,
                                            const T* __restrict__ w, int64_t n, double* __restrict__ partial, int cb)
{
    __shared__ double sred[MD_THREADS / 64][8];
    const int nc = ncols + with_ww;
    const int tid = threadIdx.x;
    const int64_t i0 = (int64_t)blockIdx.x * MD_TILE + 2 * tid, i1 = i0 + 2 * MD_THREADS;
    const bool in0 = i0 < n, in1 = i1 < n;
    const int64_t a0 = in0 ? i0 : 0, a1 = in1 ? i1 : 0;   // clamped (valid) addresses
    double2 a[8], b[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int c = cb + u;
        const T* vc = V + (int64_t)(c < ncols ? c : ncols - 1) * ldv;
        a[u] = ld2(vc + a0);
        b[u] = ld2(vc + a1);
    }
    double2 w0 = make_double2(0.0, 0.0), w1 = make_double2(0.0, 0.0);
    if (in0) w0 = ld2(w + i0);
    if (in1) w1 = ld2(w + i1);
    const double ww = w0.x * w0.x + w0.y * w0.y + w1.x * w1.x + w1.y * w1.y;
    double p[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int c = cb + u;
        const double sdot = a[u].x * w0.x + a[u].y * w0.y + b[u].x * w1.x + b[u].y * w1.y;
        p[u] = c < ncols ? sdot : (c == ncols && with_ww ? ww : 0.0);
    }
    wave_colsum8(p);
    const int lane = tid & 63, wv = tid >> 6;
    if ((lane & 7) == 0) sred[wv][lane >> 3] = p[0];
    __syncthreads();
    if (tid < 8 && cb + tid < nc) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < MD_THREADS / 64; ++k) s += sred[k][tid];
        partial[(int64_t)blockIdx.x * nc + cb + tid] = s;
    }
}

// partial[b][c] of <X_c, w> (c < ncols) and <w, w> (if with_ww), nc = ncols +
// with_ww columns in chunks of eight: grid (mdot_blocks(n), chunks x R), one
// chunk of one system per block, so every chunk's loads are in flight at
// once.  Systems r (right-hand sides sharing an operator) are addressed by
// the strides sV, sw, sP; system r is skipped when st[r] (optional) is done.
__host__ __device__ inline int mdot_chunks(int nc) { return (nc + 7) / 8; }
template <class T>
__global__ void __launch_bounds__(MD_THREADS) k_mdot_part(const T* __restrict__ V, int64_t ldv, int ncols,
                                                          int with_ww, const T* __restrict__ w, int64_t n,
                                                          double* __restrict__ partial, const GmState* __restrict__ st,
                                                          int64_t sV = 0, int64_t sw = 0, int64_t sP = 0)
{
    const int nc = ncols + with_ww, nch = mdot_chunks(nc);
    const int r = blockIdx.y / nch, cb = 8 * (blockIdx.y % nch);
    if (st && st[r].done) return;
    mdot_chunk8(V + r * sV, ldv, ncols, with_ww, w + r * sw, n, partial + r * sP, cb);
}

// out[c] = sum_b partial[b][c]; one block
__global__ void __launch_bounds__(MD_THREADS) k_mdot_fin(const double* __restrict__ partial, int nblk, int nc,
                                                         double* __restrict__ out)
{
    __shared__ double tot[MD_MAXC];
    mdot_finish(partial, nblk, nc, tot);
    for (int c = threadIdx.x; c < nc; c += MD_THREADS) out[c] = tot[c];
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

namespace pa {

// ------------------------------------------------------------------ device-resident GMRES


// One Arnoldi step after w = A v_j and the partials of <V_c, w> (c <= j)
// and <w, w> (k_mdot_part), with one classical Gram-Schmidt pass:
//   V_{j+1} = (w - V hc) / ||w - V hc||,  hc[c] = <V_c, w>,
//   ||w - V hc||^2 = <w, w> - |hc|^2 (V orthonormal).
// Grid (gm_upd_blocks(n), R), one double2 of every column per thread.
// Every block first issues the loads of w and of the first GU_COLS basis
// columns, then sums the partial rows (thread (column c, row group g) adds
// rows g, g + ng, ... of column c, the loads of up to GU_ROWS rows issued
// before the first add, so that one load latency is paid per GU_ROWS rows;
// the ng group sums are added in group order -- the same bits in every
// block), then finishes
// the update; later columns follow GU_COLS at a time, all added in column
// order.  Block 0 also rotates column j of H by the previous Givens
// rotations, makes the rotation that zeroes the subdiagonal and updates the
// residual estimate |g[j+1]|.  When the projection cancels more than 99% of
// ||w|| (where one pass would lose orthogonality) the cycle is closed at
// this column and the caller's true-residual check decides whether to
// restart.  Block 0 may set `done` while other blocks of the launch start:
// each block reads it once (either value is correct there: V_{j+1} of a
// closed cycle is never used).
constexpr int GU_THREADS = 256;
constexpr int GU_COLS = 12;    // basis columns loaded together
constexpr int GU_ROWS = 16;    // partial rows loaded together per thread
inline int64_t gm_upd_blocks(int64_t n) { return (n / 2 + GU_THREADS - 1) / GU_THREADS; }
template <class T>
__global__ void __launch_bounds__(GU_THREADS, 4) k_gm_upd(const T* __restrict__ V, int64_t ldv, int j, int m,
                                                       const T* __restrict__ w, int64_t n,
                                                       const double* __restrict__ partial, int nblk,
                                                       GmState* __restrict__ st, int64_t sV = 0, int64_t sw = 0,
                                                       int64_t sP = 0)
{
    const int r = blockIdx.y;
    V += r * sV;
    w += r * sw;
    partial += r * sP;
    st += r;
    __shared__ int sdone;
    const int tid = threadIdx.x;
    if (tid == 0) sdone = __hip_atomic_load(&st->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    if (sdone) return;
    __shared__ double s1[GM_MAXM + 2];
    __shared__ double scs[GM_MAXM], ssn[GM_MAXM];
    __shared__ double col[GM_MAXM + 2];
    __shared__ double red[GU_THREADS];
    __shared__ double sih;
    const int ncols = j + 1, nc = j + 2;
    const bool lead = blockIdx.x == 0;
    const int64_t i = ((int64_t)blockIdx.x * GU_THREADS + tid) * 2;
    const bool in = i < n;
    const int64_t ia = in ? i : 0;   // clamped (valid) address
    T* __restrict__ vnext = const_cast<T*>(V) + (int64_t)(j + 1) * ldv;
    double2 pa[GU_COLS];
#pragma unroll
    for (int u = 0; u < GU_COLS; ++u) pa[u] = ld2(V + (int64_t)(u < ncols ? u : ncols - 1) * ldv + ia);
    const double2 wv = ld2(w + ia);
    if (lead)
        for (int q = tid; q < j; q += GU_THREADS) {
            scs[q] = st->cs[q];
            ssn[q] = st->sn[q];
        }
    // final sums of the partials: ncp columns per pass (8, 16 or 32, the
    // fewest that cover nc), the 256 threads as ncp columns x ng row groups
    {
        const int ncp = nc <= 8 ? 8 : nc <= 16 ? 16 : 32, ng = GU_THREADS / ncp;
        const int cl = tid % ncp, g = tid / ncp;
        for (int c0 = 0; c0 < nc; c0 += ncp) {
            const int c = c0 + cl;
            double acc = 0.0;
            if (c < nc)
                for (int b0 = g; b0 < nblk; b0 += GU_ROWS * ng) {
                    // all GU_ROWS loads issued before the first add (rows
                    // past nblk read the last row and add zero)
                    const double* pc = partial + c;
                    double v[GU_ROWS];
#pragma unroll
                    for (int u = 0; u < GU_ROWS; ++u) {
                        const int b = b0 + u * ng;
                        v[u] = pc[(b < nblk ? b : nblk - 1) * nc];
                    }
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int u = 0; u < GU_ROWS; ++u) acc += b0 + u * ng < nblk ? v[u] : 0.0;
                }
            red[tid] = acc;
            __syncthreads();
            if (tid < ncp && c0 + tid < nc) {
                double sum = 0.0;
                for (int gg = 0; gg < ng; ++gg) sum += red[gg * ncp + tid];
                s1[c0 + tid] = sum;
            }
            __syncthreads();
        }
    }
    if (tid == 0) {
        double proj = 0.0;
        for (int q = 0; q < ncols; ++q) proj += s1[q] * s1[q];
        const double ww = s1[ncols], rem = ww - proj;
        const double hn = rem > 0.0 ? sqrt(rem) : 0.0;
        sih = hn > 0.0 ? 1.0 / hn : 0.0;
        if (lead) {
            const bool close = !(rem > 1e-4 * ww);
            for (int q = 0; q < ncols; ++q) col[q] = s1[q];
            col[j + 1] = hn;
            for (int q = 0; q < j; ++q) {
                const double a = col[q], b = col[q + 1];
                col[q] = scs[q] * a + ssn[q] * b;
                col[q + 1] = -ssn[q] * a + scs[q] * b;
            }
            const double a = col[j], b = col[j + 1];
            const double rr = sqrt(a * a + b * b);
            const double c = a / rr, sgn = b / rr;
            col[j] = rr;
            col[j + 1] = 0.0;
            const double gj = st->g[j];
            const double gj1 = -sgn * gj;
            st->cs[j] = c;
            st->sn[j] = sgn;
            st->g[j] = c * gj;
            st->g[j + 1] = gj1;
            const double res = fabs(gj1);
            st->res = res;
            if (!(res > st->tol) || hn == 0.0 || close || !(res == res)) {
                st->its = j + 1;
                __hip_atomic_store(&st->done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
    __syncthreads();
    if (lead)
        for (int q = tid; q <= j + 1; q += GU_THREADS) st->H[q * m + j] = col[q];
    // V_{j+1}
    double sx = 0.0, sy = 0.0;
#pragma unroll
    for (int u = 0; u < GU_COLS; ++u) {
        const double h = u < ncols ? s1[u] : 0.0;
        sx += h * pa[u].x;
        sy += h * pa[u].y;
    }
    for (int c0 = GU_COLS; c0 < ncols; c0 += GU_COLS) {
        double2 a[GU_COLS];
#pragma unroll
        for (int u = 0; u < GU_COLS; ++u) a[u] = ld2(V + (int64_t)(c0 + u < ncols ? c0 + u : ncols - 1) * ldv + ia);
#pragma unroll
        for (int u = 0; u < GU_COLS; ++u) {
            const double h = c0 + u < ncols ? s1[c0 + u] : 0.0;
            sx += h * a[u].x;
            sy += h * a[u].y;
        }
    }
    const double ih = sih;
    if (in) st2(vnext + i, make_double2((wv.x - sx) * ih, (wv.y - sy) * ih));
}

// start of a cycle from the partials of <r, r>: beta = ||r||, g = beta e_1,
// V_0 = r / beta (every block sums the partials in the same order; block 0
// writes the state)
constexpr int GM_RMAX = 8;   // systems per launch
struct GmTol { double t[GM_RMAX]; };
template <class T>
__global__ void __launch_bounds__(MD_THREADS) k_gm_begin(const T* __restrict__ r, T* __restrict__ v0,
                                                         int64_t n, const double* __restrict__ partial, int nblk,
                                                         GmTol tols, GmState* __restrict__ st, int64_t sr = 0,
                                                         int64_t sV = 0, int64_t sP = 0)
{
    const int sys = blockIdx.y;
    r += sys * sr;
    v0 += sys * sV;
    partial += sys * sP;
    st += sys;
    const double tol = tols.t[sys];
    __shared__ double tot[1];
    mdot_finish(partial, nblk, 1, tot);
    const double beta = sqrt(tot[0]);
    const double ib = beta > 0.0 ? 1.0 / beta : 0.0;
    if (blockIdx.x == 0) {
        for (int i = threadIdx.x; i <= GM_MAXM; i += blockDim.x) st->g[i] = i == 0 ? beta : 0.0;
        if (threadIdx.x == 0) {
            st->res = beta;
            st->tol = tol;
            st->its = 0;
            st->done = (beta > tol) ? 0 : 1;
        }
    }
    const int64_t i0 = (int64_t)blockIdx.x * MD_TILE + 2 * threadIdx.x, i1 = i0 + 2 * MD_THREADS;
    if (i0 < n) {
        const double2 ri = ld2(r + i0);
        st2(v0 + i0, make_double2(ri.x * ib, ri.y * ib));
    }
    if (i1 < n) {
        const double2 ri = ld2(r + i1);
        st2(v0 + i1, make_double2(ri.x * ib, ri.y * ib));
    }
}

// y = R^{-1} g for the first k columns (k = its if done else m); R is
// staged in LDS by all lanes, one lane back-substitutes
__global__ void __launch_bounds__(256) k_gm_solve(int m, GmState* __restrict__ st)
{
    st += blockIdx.x;   // one block per system
    __shared__ double R[GM_MAXM * GM_MAXM];
    __shared__ double yy[GM_MAXM];
    const int k = st->done ? st->its : m;
    for (int t = threadIdx.x; t < k * k; t += blockDim.x) R[t] = st->H[(t / k) * m + (t % k)];
    for (int t = threadIdx.x; t < k; t += blockDim.x) yy[t] = st->g[t];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int i = k - 1; i >= 0; --i) {
            double s = yy[i];
            for (int c = i + 1; c < k; ++c) s -= R[i * k + c] * yy[c];
            yy[i] = s / R[i * k + i];
        }
    __syncthreads();
    for (int t = threadIdx.x; t < m; t += blockDim.x) st->y[t] = t < k ? yy[t] : 0.0;
}

// out = sum_{c<m} y[c] V_c   (y is zero beyond the cycle's length)
template <class T>
__global__ void k_gm_combine(const T* __restrict__ V, int64_t ldv, int m, double* __restrict__ out, int64_t n,
                             const GmState* __restrict__ st, int64_t sV = 0, int64_t sOut = 0)
{
    V += blockIdx.y * sV;
    out += blockIdx.y * sOut;
    st += blockIdx.y;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int k = st->done ? st->its : m;
    double s = 0.0;
    for (int c = 0; c < k; ++c) s += st->y[c] * V[(int64_t)c * ldv + i];
    out[i] = s;
}

}  // namespace pa

namespace pa {

// ------------------------------------------------------------------ preconditioned stage operator
// A = M - c J with the block-Jacobi factor P = blockdiag(A) folded in:
//   Ahat = A P^{-1}:  Ahat_KK = I,  Ahat_{K,nb} = -c J_{K,nb} P_nb^{-1}.
// Forward solves (right preconditioning):   Ahat y = b,  x = P^{-1} y.
// Transposed solves (left preconditioning): Ahat^T x = P^{-T} b.
// Only the three off-diagonal blocks of a row are streamed per iteration.

// P (diagonal blocks of A) and P^{-1} by Gauss-Jordan elimination with
// partial pivoting (largest magnitude, lowest row on ties), one wave per
// block, the block held in registers: lane i owns row i.
//  - step k: the pivot is the largest |a[i][k]| over the rows not yet
//    pivotal, found by a butterfly of cross-lane exchanges; the pivot row is
//    broadcast from its lane (readlane) and the in-place Gauss-Jordan update
//    runs on every lane at once (row p: a[p][:] /= a[p][k] with a[p][k] =
//    1 / pivot; row i != p: a[i][:] -= a[i][k] a[p][:], a[i][k] =
//    -a[i][k] / pivot);
//  - with rows taken in the pivot order p_0, p_1, ... this inverts the row-
//    permuted block, so lane p_k ends with row k of P^{-1} with its columns
//    in pivot order (entry c belongs to column p_c); the rows are put back
//    in place through LDS and stored coalesced.
__device__ __forceinline__ double bcast_lane(double x, int src)
{
    const long long v = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)v, src);
    const int hi = __builtin_amdgcn_readlane((int)(v >> 32), src);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <int NP>
__global__ void __launch_bounds__(64) k_blockprep(int Ne, const double* __restrict__ area, const double* __restrict__ mh,
                                                  const double* __restrict__ J, double c, double* __restrict__ Pd,
                                                  double* __restrict__ Pinv, int* __restrict__ status)
{
    constexpr int B = 4 * NP, BB = B * B;
    static_assert(B <= 64, "one lane per row");
    __shared__ double t[B][B + 1];
    __shared__ int pc[B];
    const int K = blockIdx.x, lane = threadIdx.x;
    const double* src = J + (int64_t)K * 4 * BB;
    const double s2 = 2.0 * area[K];
    double* pd = Pd + (int64_t)K * BB;
    // every load (the Jacobian block's and the mass entries') issued before
    // the first use
    constexpr int NL = (BB + 63) / 64;
    double sv[NL], mv[NL];
#pragma unroll
    for (int u = 0; u < NL; ++u) {
        const int q = lane + 64 * u < BB ? lane + 64 * u : BB - 1;
        sv[u] = src[q];
        mv[u] = mh[(q / B >> 2) * NP + (q % B >> 2)];
    }
#pragma unroll
    for (int u = 0; u < NL; ++u) {
        const int q = lane + 64 * u;
        if (q < BB) {
            const int i = q / B, j = q % B;
            const double mm = ((i & 3) == (j & 3)) ? s2 * mv[u] : 0.0;
            const double v = mm - c * sv[u];
            t[i][j] = v;
            pd[q] = v;
        }
    }
    __syncthreads();
    const int row = lane < B ? lane : B - 1;
    double a[B];
#pragma unroll
    for (int j = 0; j < B; ++j) a[j] = t[row][j];
    bool used = lane >= B;
    int kpos = 0;
    bool singular = false;
#pragma clang loop unroll(full)
    for (int k = 0; k < B; ++k) {
        double v = used ? -1.0 : fabs(a[k]);
        int idx = lane;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const double ov = __shfl_xor(v, off, 64);
            const int oi = __shfl_xor(idx, off, 64);
            if (ov > v || (ov == v && oi < idx)) { v = ov; idx = oi; }
        }
        const int p = __builtin_amdgcn_readfirstlane(idx);
        singular = singular || v == 0.0;
        const double ipv = 1.0 / bcast_lane(a[k], p);
        const bool me = lane == p;
        const double f = a[k];
        const double g = me ? 0.0 : f * ipv;   // multiple of the (unscaled) pivot row taken away
        const double sc = me ? ipv : 1.0;      // the pivot row itself is scaled
#pragma clang loop unroll(full)
        for (int j = 0; j < B; ++j) {
            if (j == k) continue;
            const double apj = bcast_lane(a[j], p);
            a[j] = (a[j] - g * apj) * sc;
        }
        a[k] = me ? ipv : -f * ipv;
        if (me) { used = true; kpos = k; }
        if (lane == 0) pc[k] = p;
    }
    if (lane == 0 && singular) status[0] = 1;
    __syncthreads();
    if (lane < B)
#pragma unroll
        for (int cc = 0; cc < B; ++cc) t[kpos][pc[cc]] = a[cc];
    __syncthreads();
    double* dst = Pinv + (int64_t)K * BB;
    for (int q = lane; q < BB; q += 64) dst[q] = t[q / B][q % B];
}

// ------------------------------------------------------------------ one-workgroup stage solve
// For meshes small enough that every kernel of an iteration is dominated by
// its launch (N_u up to WG_MAXNU), the whole stage solve -- GMRES(m) on
// Ahat y = b (or Ahat^T y = b) with restarts and the true-residual check --
// runs in one workgroup of WG_THREADS threads per system (grid = systems,
// strides sb, sy, sV, sw between them), with no kernel boundary inside it.
// The same algorithm as the multi-kernel solve: x0 = 0, one classical
// Gram-Schmidt pass per iteration (a column whose projection cancels more
// than 99% of ||w|| closes the cycle), Givens rotations, a cycle accepted on
// its true residual ||b - Ahat y|| <= 2 tol with tol = rtol ||b||, at most
// maxit iterations.  Thread t owns rows t, t + WG_THREADS, ...; every sum
// over rows is a fixed-order block reduction (bitwise reproducible).  The
// apply reads the three stored blocks of a row (transposed: the neighbours'
// twin blocks, by column) from L2, where the operator and the basis stay
// across iterations at these sizes.
constexpr int WG_THREADS = 512;
constexpr int WG_MAXNU = 16384;
constexpr int WG_MAXM = 64;
struct WgStatus {
    int its;        // GMRES iterations over all cycles
    int conv;       // 1: converged; 0: iteration limit; -1: not finite
    double res;     // final true residual norm
};

// fixed-order sum over the block of one value per thread; every thread gets it
__device__ __forceinline__ double wg_sum(double v, double* sred)
{
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    __syncthreads();
    if (lane == 0) sred[wv] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < WG_THREADS / 64; ++k) s += sred[k];
    return s;
}

template <int NP>
__device__ __forceinline__ void wg_apply(int Ne, const int32_t* __restrict__ enb, const int8_t* __restrict__ etw,
                                         const double* __restrict__ Ah, int tr, const double* x, double* out)
{
    constexpr int B = 4 * NP, BB = B * B;
    const int64_t Nu = (int64_t)Ne * B;
    for (int64_t rr = threadIdx.x; rr < Nu; rr += WG_THREADS) {
        const int K = (int)(rr / B), i = (int)(rr % B);
        double acc = x[rr];
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            const int nb = enb[3 * K + f];
            if (nb < 0) continue;
            const double* xn = x + (int64_t)nb * B;
            if (!tr) {
                const double* blk = Ah + ((int64_t)K * 3 + f) * BB + (int64_t)i * B;
#pragma unroll
                for (int j = 0; j < B; ++j) acc += blk[j] * xn[j];
            } else {
                const double* blk = Ah + ((int64_t)nb * 3 + etw[3 * K + f]) * BB + i;
#pragma unroll
                for (int j = 0; j < B; ++j) acc += blk[(int64_t)j * B] * xn[j];
            }
        }
        out[rr] = acc;
    }
}

template <int NP>
__global__ void __launch_bounds__(WG_THREADS) k_stage_gmres_wg(int Ne, const int32_t* __restrict__ enb,
                                                               const int8_t* __restrict__ etw,
                                                               const double* __restrict__ Ah, int tr,
                                                               const double* __restrict__ b, double* __restrict__ y,
                                                               double* __restrict__ V, double* __restrict__ w,
                                                               int m, int maxit, double rtol, WgStatus* status,
                                                               int64_t sb, int64_t sy, int64_t sV, int64_t sw)
{
    constexpr int B = 4 * NP;
    const int64_t Nu = (int64_t)Ne * B;
    const int sys = blockIdx.x, tid = threadIdx.x;
    b += sys * sb;
    y += sys * sy;
    V += sys * sV;
    w += sys * sw;
    status += sys;
    __shared__ double sred[WG_THREADS / 64];
    __shared__ double red[WG_THREADS / 64][33];
    __shared__ double H[(WG_MAXM + 1) * WG_MAXM];
    __shared__ double g[WG_MAXM + 1], cs[WG_MAXM], sn[WG_MAXM], hc[WG_MAXM + 2], yc[WG_MAXM], col[WG_MAXM + 2];
    __shared__ double s_ih;
    __shared__ int s_done;
    double bb = 0.0;
    for (int64_t rr = tid; rr < Nu; rr += WG_THREADS) {
        const double v = b[rr];
        bb += v * v;
        y[rr] = 0.0;
    }
    const double bn = sqrt(wg_sum(bb, sred));
    const double tol = rtol * bn;
    int total = 0, conv = 0;
    double rn = bn;
    if (!(bn > 0.0)) {
        if (tid == 0) { status->its = 0; status->conv = bn == 0.0 ? 1 : -1; status->res = bn; }
        return;
    }
    // r = b - Ahat y lives in w at the start of each cycle (y = 0: r = b)
    for (int64_t rr = tid; rr < Nu; rr += WG_THREADS) w[rr] = b[rr];
    for (;;) {
        // cycle start: V_0 = r / |r|, g = |r| e_1
        const double ib = 1.0 / rn;
        for (int64_t rr = tid; rr < Nu; rr += WG_THREADS) V[rr] = w[rr] * ib;
        if (tid == 0) {
            g[0] = rn;
            s_done = 0;
        }
        __syncthreads();
        int its = m;
        for (int j = 0; j < m; ++j) {
            const double* vj = V + (int64_t)j * Nu;
            wg_apply<NP>(Ne, enb, etw, Ah, tr, vj, w);
            // <V_c, w> (c <= j) and <w, w>: each thread reads only its own rows of w
            const int nc = j + 2;
            for (int c0 = 0; c0 < nc; c0 += 32) {
                double p[MD_GROUP];
#pragma unroll
                for (int u = 0; u < MD_GROUP; ++u) p[u] = 0.0;
                for (int64_t rr = tid; rr < Nu; rr += WG_THREADS) {
                    const double wv = w[rr];
#pragma unroll
                    for (int u = 0; u < MD_GROUP; ++u) {
                        const int c = c0 + u;
                        if (c <= j) p[u] += V[(int64_t)c * Nu + rr] * wv;
                        else if (c == j + 1) p[u] += wv * wv;
                    }
                }
                wave_colsum32(p);
                const int lane = tid & 63, wv = tid >> 6;
                if ((lane & 1) == 0) red[wv][lane >> 1] = p[0];
                __syncthreads();
                if (tid < 32 && c0 + tid < nc) {
                    double sum = 0.0;
#pragma unroll
                    for (int k = 0; k < WG_THREADS / 64; ++k) sum += red[k][tid];
                    hc[c0 + tid] = sum;
                }
                __syncthreads();
            }
            if (tid == 0) {
                double proj = 0.0;
                for (int q = 0; q <= j; ++q) proj += hc[q] * hc[q];
                const double ww = hc[j + 1], rem = ww - proj;
                const double hn = rem > 0.0 ? sqrt(rem) : 0.0;
                s_ih = hn > 0.0 ? 1.0 / hn : 0.0;
                const bool close = !(rem > 1e-4 * ww);
                for (int q = 0; q <= j; ++q) col[q] = hc[q];
                col[j + 1] = hn;
                for (int q = 0; q < j; ++q) {
                    const double a = col[q], bq = col[q + 1];
                    col[q] = cs[q] * a + sn[q] * bq;
                    col[q + 1] = -sn[q] * a + cs[q] * bq;
                }
                const double a = col[j], bq = col[j + 1];
                const double rr2 = sqrt(a * a + bq * bq);
                cs[j] = a / rr2;
                sn[j] = bq / rr2;
                col[j] = rr2;
                for (int q = 0; q <= j; ++q) H[q * WG_MAXM + j] = col[q];
                const double gj = g[j];
                g[j] = cs[j] * gj;
                g[j + 1] = -sn[j] * gj;
                const double res = fabs(g[j + 1]);
                if (!(res > tol) || hn == 0.0 || close || !(res == res)) s_done = 1;
            }
            __syncthreads();
            const bool done = s_done != 0;
            if (!done) {
                // V_{j+1} = (w - V hc) ih (V holds m + 1 columns)
                const double ih = s_ih;
                double* vn = V + (int64_t)(j + 1) * Nu;
                for (int64_t rr = tid; rr < Nu; rr += WG_THREADS) {
                    double sacc = 0.0;
                    for (int c = 0; c <= j; ++c) sacc += hc[c] * V[(int64_t)c * Nu + rr];
                    vn[rr] = (w[rr] - sacc) * ih;
                }
            }
            __syncthreads();
            if (done) {
                its = j + 1;
                break;
            }
        }
        // y += V R^{-1} g over the cycle's columns
        if (tid == 0)
            for (int q = its - 1; q >= 0; --q) {
                double sacc = g[q];
                for (int c = q + 1; c < its; ++c) sacc -= H[q * WG_MAXM + c] * yc[c];
                yc[q] = sacc / H[q * WG_MAXM + q];
            }
        __syncthreads();
        for (int64_t rr = tid; rr < Nu; rr += WG_THREADS) {
            double sacc = 0.0;
            for (int c = 0; c < its; ++c) sacc += yc[c] * V[(int64_t)c * Nu + rr];
            y[rr] += sacc;
        }
        __syncthreads();
        total += its;
        // true residual r = b - Ahat y, into w
        wg_apply<NP>(Ne, enb, etw, Ah, tr, y, w);
        double rr2 = 0.0;
        for (int64_t rr = tid; rr < Nu; rr += WG_THREADS) {
            const double v = b[rr] - w[rr];
            w[rr] = v;
            rr2 += v * v;
        }
        rn = sqrt(wg_sum(rr2, sred));
        if (!(rn == rn)) { conv = -1; break; }
        if (rn <= 2.0 * tol) { conv = 1; break; }
        if (total >= maxit) break;
        __syncthreads();
    }
    if (tid == 0) {
        status->its = total;
        status->conv = conv;
        status->res = rn;
    }
}

template <int NP>
__global__ void __launch_bounds__(64) k_form_ahat_mfma(int Ne, const int32_t* __restrict__ enb,
                                                       const double* __restrict__ J, double c,
                                                       const double* __restrict__ Pinv, double* __restrict__ Ah)
{
    constexpr int B = 4 * NP, BB = B * B, T = (B + 15) / 16, KS = B / 4;
    __shared__ double sj[B][B + 1];
    __shared__ double sp[B][B + 1];
    const int K = blockIdx.x / 3, f = blockIdx.x % 3, lane = threadIdx.x;
    const int nb = enb[3 * K + f];
    double* dst = Ah + ((int64_t)K * 3 + f) * BB;
    if (nb < 0) {
        for (int t = lane; t < BB; t += 64) dst[t] = 0.0;
        return;
    }
    const double* js = J + ((int64_t)K * 4 + 1 + f) * BB;
    const double* ps = Pinv + (int64_t)nb * BB;
    // both blocks as double2 (B is even: a pair never straddles rows), every
    // load issued before the first LDS store
    constexpr int H2 = BB / 2, NL = (H2 + 63) / 64;
    double2 vj[NL], vp[NL];
#pragma unroll
    for (int u = 0; u < NL; ++u) {
        const int t2 = lane + 64 * u < H2 ? lane + 64 * u : H2 - 1;
        vj[u] = reinterpret_cast<const double2*>(js)[t2];
        vp[u] = reinterpret_cast<const double2*>(ps)[t2];
    }
#pragma unroll
    for (int u = 0; u < NL; ++u) {
        const int t2 = lane + 64 * u;
        if (t2 < H2) {
            const int i = 2 * t2 / B, j = 2 * t2 % B;
            sj[i][j] = -c * vj[u].x;
            sj[i][j + 1] = -c * vj[u].y;
            sp[i][j] = vp[u].x;
            sp[i][j + 1] = vp[u].y;
        }
    }
    __syncthreads();
    const int li = lane % 16, lk = lane / 16;
    for (int ti = 0; ti < T; ++ti) {
        const int row = ti * 16 + li;
        for (int tj = 0; tj < T; ++tj) {
            const int colb = tj * 16 + li;
            mf_d4 acc = { 0.0, 0.0, 0.0, 0.0 };
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const int kk = ks * 4 + lk;
                const double a = row < B ? sj[row][kk] : 0.0;
                const double b = colb < B ? sp[kk][colb] : 0.0;
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
            }
            const int col = tj * 16 + li;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = ti * 16 + lk + 4 * r;
                if (i < B && col < B) dst[i * B + col] = acc[r];
            }
        }
    }
}

template <int NP>
__global__ void __launch_bounds__(64) k_form_ahat(int Ne, const int32_t* __restrict__ enb, const double* __restrict__ J,
                                                  double c, const double* __restrict__ Pinv, double* __restrict__ Ah)
{
    constexpr int B = 4 * NP, BB = B * B;
    __shared__ double sj[B][B + 1];
    __shared__ double sp[B][B + 1];
    const int K = blockIdx.x / 3, f = blockIdx.x % 3, lane = threadIdx.x;
    const int nb = enb[3 * K + f];
    double* dst = Ah + ((int64_t)K * 3 + f) * BB;
    if (nb < 0) {
        for (int t = lane; t < BB; t += 64) dst[t] = 0.0;
        return;
    }
    const double* js = J + ((int64_t)K * 4 + 1 + f) * BB;
    const double* ps = Pinv + (int64_t)nb * BB;
    for (int t = lane; t < BB; t += 64) {
        sj[t / B][t % B] = -c * js[t];
        sp[t / B][t % B] = ps[t];
    }
    __syncthreads();
    for (int t = lane; t < BB; t += 64) {
        int i = t / B, j = t % B;
        double s = 0.0;
#pragma unroll 8
        for (int k = 0; k < B; ++k) s += sj[i][k] * sp[k][j];
        dst[t] = s;
    }
}

// ------------------------------------------------------------------ low-precision stage operator
// Storage formats of the inner operator of the mixed-precision solve: FP32,
// or BF16 (the upper 16 bits of an FP32, rounded to nearest even through
// FP32).  Arithmetic and accumulation are FP32 in both.
struct bf16_t { uint16_t b; };
__device__ __forceinline__ float lo_to_f(float v) { return v; }
__device__ __forceinline__ float lo_to_f(bf16_t v) { return __uint_as_float((uint32_t)v.b << 16); }
__device__ __forceinline__ void f_to_lo(double v, float& o) { o = (float)v; }
__device__ __forceinline__ void f_to_lo(double v, bf16_t& o)
{
    const uint32_t u = __float_as_uint((float)v);
    if ((u & 0x7f800000u) == 0x7f800000u) {           // Inf / NaN: keep class, quiet NaN
        o.b = (uint16_t)((u >> 16) | ((u & 0x007fffffu) ? 0x40u : 0u));
        return;
    }
    o.b = (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

// dst = lo(src), n entries
template <class TM>
__global__ void k_to_lo(const double* __restrict__ src, TM* __restrict__ dst, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) f_to_lo(src[i], dst[i]);
}

// y = x + Ahat_lo x or y = x + Ahat_lo^T x in FP32 (as k_ahat_apply, with
// 16-byte loads of 4 FP32 or 8 BF16 entries)
template <int NP, class TM>
__global__ void __launch_bounds__(64) k_ahat_apply_lo(int Ne, const int32_t* __restrict__ enb,
                                                      const int8_t* __restrict__ etw, const TM* __restrict__ Ah,
                                                      const float* __restrict__ x, float* __restrict__ y, int trans,
                                                      const int* __restrict__ skip)
{
    constexpr int B = 4 * NP, BB = B * B;
    constexpr int EPL = 16 / sizeof(TM);              // entries per 16-byte load
    constexpr int H = BB / EPL;                       // loads per block
    constexpr int PER = (H + 63) / 64;
    __shared__ float sblk[3][B][B + 1];
    __shared__ float sx[3][B];
    if (skip && *skip) return;
    const int K = blockIdx.x, lane = threadIdx.x;
    int nbs[3];
    const uint4* src[3];
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        int nb = enb[3 * K + f];
        nbs[f] = nb;
        src[f] = nullptr;
        if (nb >= 0) {
            int64_t blk = trans ? (int64_t)nb * 3 + etw[3 * K + f] : (int64_t)K * 3 + f;
            src[f] = reinterpret_cast<const uint4*>(Ah + blk * BB);
        }
    }
    uint4 v[3][PER];
#pragma unroll
    for (int f = 0; f < 3; ++f)
#pragma unroll
        for (int r = 0; r < PER; ++r) {
            int t = lane + 64 * r;
            if (src[f] && t < H) v[f][r] = src[f][t];
        }
#pragma unroll
    for (int f = 0; f < 3; ++f)
        if (nbs[f] >= 0 && lane < B) sx[f][lane] = x[(int64_t)nbs[f] * B + lane];
#pragma unroll
    for (int f = 0; f < 3; ++f)
#pragma unroll
        for (int r = 0; r < PER; ++r) {
            int t = lane + 64 * r;
            if (src[f] && t < H) {
                const TM* e8 = reinterpret_cast<const TM*>(&v[f][r]);
#pragma unroll
                for (int q = 0; q < EPL; ++q) {
                    int e = EPL * t + q;
                    sblk[f][e / B][e % B] = lo_to_f(e8[q]);
                }
            }
        }
    __syncthreads();
    if (lane < B) {
        float acc = x[(int64_t)K * B + lane];
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            if (nbs[f] < 0) continue;
            float a = 0.0f;
            if (!trans) {
#pragma unroll 8
                for (int j = 0; j < B; ++j) a += sblk[f][lane][j] * sx[f][j];
            } else {
#pragma unroll 8
                for (int i = 0; i < B; ++i) a += sblk[f][i][lane] * sx[f][i];
            }
            acc += a;
        }
        y[(int64_t)K * B + lane] = acc;
    }
}

// Forward apply y = x + Ahat x for any storage type TM (double, float,
// bf16_t) with TV vectors; accumulation in TV (FP64 for the FP64 operator,
// FP32 otherwise).  One wave per block row.  A task is Q consecutive 16-byte
// chunks of one row of a row-major block (Q chosen so that a task never
// straddles rows and holds at most 8 entries): the lane loads them with Q
// coalesced 16-byte loads (all tasks of the three blocks before any
// arithmetic), multiplies them by the matching entries of x in registers and
// leaves one partial per task in LDS, stored task-major with a padded stride
// (conflict-free both ways).  Lane i then adds the partials of row i in task
// order (B / (Q EPL) per block, 5 at p = 3 for every storage type).
template <class TA> __device__ __forceinline__ TA to_acc(double v) { return (TA)v; }
template <class TA> __device__ __forceinline__ TA to_acc(float v) { return (TA)v; }
template <class TA> __device__ __forceinline__ TA to_acc(bf16_t v) { return (TA)lo_to_f(v); }

template <int B, int EPL>
constexpr int fwd_chunks_per_task()
{
    return (8 % EPL == 0 && B % 8 == 0) ? 8 / EPL : (B % (2 * EPL) == 0 && 2 * EPL <= 8 ? 2 : 1);
}

// tile shape of the forward apply: chunks per task Q (0 = the default above);
// a context times the valid shapes on its first stored operator and keeps
// the fastest (ahat_fwd_valid tells which Q fit the block size)
template <int NP, class TM>
constexpr bool ahat_fwd_valid(int Q)
{
    return (4 * NP) % (int)(16 / sizeof(TM) * Q) == 0 && (int)(16 / sizeof(TM)) * Q <= 8;
}

// Per-element face tables of the stage-operator applies, one int4 per
// element so that a wave reads them with one scalar load:
//   fwd: {nb_0, nb_1, nb_2, mask}, nb_f the neighbour across face f;
//   tr:  {b_0, b_1, b_2, mask}, b_f = 3 nb_f + twin_f, the neighbour's block
//        that points back at this element;
// bit f of mask is set for an interior face.  For a boundary face nb_f is the
// element itself and b_f its own slot f, whose stored block is zero: every
// load of the applies then has a valid address and is issued without a
// branch, and the face's contribution is removed by a zero weight.

// Forward apply y = x + Ahat x (Ahat's diagonal blocks are the identity):
// y_i = x_i + sum_f sum_j A_f[i][j] x_nb_f[j] over the three stored
// off-diagonal blocks of block row K.  Each block is split into tasks of Q
// 16-byte chunks lying in one row; lane l holds tasks l, l + 64, ... of the
// three blocks in registers (every load issued before any arithmetic, no
// matrix entry through LDS), leaves one partial per task in LDS, and lane i
// adds row i's partials to x_i.  With Ahp (optional, in every apply
// kernel) the blocks' address is read from device memory at the start: a
// launch captured once in a graph then serves whichever stored operator the
// slot names when it is replayed.
template <int NP, class TM, class TV, int QT = 0>
__global__ void __launch_bounds__(64) k_ahat_fwd(int Ne, const int4* __restrict__ nb4, const TM* __restrict__ Ah,
                                                 const TV* __restrict__ x, TV* __restrict__ y,
                                                 const int* __restrict__ skip, const TM* const* __restrict__ Ahp = nullptr)
{
    constexpr int B = 4 * NP, BB = B * B;
    constexpr int EPL = 16 / sizeof(TM);              // entries per 16-byte chunk
    static_assert(B % EPL == 0, "a chunk must not straddle rows");
    constexpr int Q = QT > 0 ? QT : fwd_chunks_per_task<B, EPL>();  // chunks per task
    constexpr int EPT = Q * EPL;                      // entries per task
    static_assert(B % EPT == 0, "a task must not straddle rows");
    constexpr int H = BB / EPT, TPR = B / EPT;        // tasks per block / per row
    constexpr int PER = (H + 63) / 64;
    __shared__ TV sp[3][TPR][B + 1];
    __shared__ TV sx[3][B];
    if (skip && *skip) return;
    if (Ahp) Ah = *Ahp;
    const int K = blockIdx.x, lane = threadIdx.x;
    const int4 t4 = nb4[K];
    int nbs[3];
    const uint4* src[3];
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        nbs[f] = (t4.w >> f) & 1 ? (f == 0 ? t4.x : f == 1 ? t4.y : t4.z) : -1;
        src[f] = nbs[f] >= 0 ? reinterpret_cast<const uint4*>(Ah + ((int64_t)K * 3 + f) * BB) : nullptr;
    }
    // own entry of x, needed only at the end, loaded with the others
    const TV xo = x[(int64_t)K * B + lane % B];
    uint4 v[3][PER][Q];
#pragma unroll
    for (int f = 0; f < 3; ++f)
#pragma unroll
        for (int r = 0; r < PER; ++r) {
            const int t = lane + 64 * r;
            if (src[f] && t < H)
#pragma unroll
                for (int q = 0; q < Q; ++q) v[f][r][q] = src[f][t * Q + q];
        }
#pragma unroll
    for (int f = 0; f < 3; ++f)
        if (nbs[f] >= 0 && lane < B) sx[f][lane] = x[(int64_t)nbs[f] * B + lane];
    __syncthreads();
#pragma unroll
    for (int f = 0; f < 3; ++f)
#pragma unroll
        for (int r = 0; r < PER; ++r) {
            const int t = lane + 64 * r;
            if (src[f] && t < H) {
                const int i = t / TPR, c = t % TPR;
                TV p = 0;
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    const TM* e = reinterpret_cast<const TM*>(&v[f][r][q]);
#pragma unroll
                    for (int u = 0; u < EPL; ++u) p += to_acc<TV>(e[u]) * sx[f][c * EPT + q * EPL + u];
                }
                sp[f][c][i] = p;
            }
        }
    __syncthreads();
    if (lane < B) {
        TV acc = xo;
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            if (nbs[f] < 0) continue;
#pragma unroll
            for (int c = 0; c < TPR; ++c) acc += sp[f][c][lane];
        }
        y[(int64_t)K * B + lane] = acc;
    }
}

// Transposed apply y = x + Ahat^T x: row K of Ahat^T takes, for each
// neighbour nb across face f, the block of nb that points back at K (slot
// twin) transposed, so y[j] = x[j] + sum_f sum_i A_f[i][j] x_nb_f[i].
// Lanes 0..59 of the wave are (row group g, column chunk c) with G = 60 /
// CPR groups: lane (g, c) loads chunk c of rows g, g + G, g + 2G, ... of the
// three blocks -- for every row step the 60 lanes read 60 consecutive
// 16-byte chunks -- and sums over the faces and its rows in registers.  The
// G partials of a column chunk are added by lane (0, c) with cross-lane
// reads in group order, and that lane writes the chunk's EPL entries of y.
// One barrier: the neighbours' entries of x are staged in LDS.
template <int NP, class TM, class TV, int R>
__device__ __forceinline__ void ahat_tr_body(int K, const int4* __restrict__ tb4, const TM* __restrict__ Ah,
                                             const TV* __restrict__ x, int64_t sx, TV* __restrict__ y, int64_t sy)
{
    constexpr int B = 4 * NP, BB = B * B;
    constexpr int EPL = 16 / sizeof(TM);
    static_assert(B % EPL == 0, "a chunk must not straddle rows");
    constexpr int CPR = B / EPL;
    static_assert(60 % CPR == 0, "row groups must tile 60 lanes");
    constexpr int G = 60 / CPR, RPL = (B + G - 1) / G;
    __shared__ TV sxs[R][3][B + G];                  // rows B.. B+G-1 zero: the last row step needs no test
    const int lane = threadIdx.x;
    const int c = lane % CPR, g = lane < 60 ? lane / CPR : 0;   // lanes 60..63 repeat group 0 (unused)
    const int4 t4 = tb4[K];
    const int blk[3] = { t4.x, t4.y, t4.z };
    const int mask = t4.w;
    const int li = lane % B;
    // x first, into registers (staging it in LDS before the barrier then
    // waits for these loads only); the own chunk for lanes (0, c)
    TV xo[R][EPL], xn[R][3];
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
        for (int q = 0; q < EPL; ++q) xo[r][q] = x[r * sx + (int64_t)K * B + c * EPL + q];
#pragma unroll
        for (int f = 0; f < 3; ++f) xn[r][f] = x[r * sx + (int64_t)(blk[f] / 3) * B + li];
    }
    asm volatile("" ::: "memory");   // compiler-only fence: the loads of x stay ahead of the block loads
    uint4 v[3][RPL];
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        const uint4* src = reinterpret_cast<const uint4*>(Ah + (int64_t)blk[f] * BB);
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
            const int i = g + G * k < B ? g + G * k : B - 1;
            v[f][k] = src[i * CPR + c];
        }
    }
    // every lane stores (lanes past the block repeat the value of lane
    // li), so no branch lets the compiler sink the loads of x past the
    // block loads
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
        for (int f = 0; f < 3; ++f) sxs[r][f][li] = xn[r][f];
        if (lane < G)
#pragma unroll
            for (int f = 0; f < 3; ++f) sxs[r][f][B + lane] = TV(0);
    }
    __syncthreads();
    TV p[R][EPL];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int q = 0; q < EPL; ++q) p[r][q] = 0;
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        // interior faces only (a uniform branch, which also keeps the LDS
        // reads of one face from being hoisted ahead of the others'
        // arithmetic and held in registers all at once)
        if (!((mask >> f) & 1)) continue;
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
            const int i = g + G * k;
            const TM* e = reinterpret_cast<const TM*>(&v[f][k]);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const TV xi = sxs[r][f][i];
#pragma unroll
                for (int q = 0; q < EPL; ++q) p[r][q] += to_acc<TV>(e[q]) * xi;
            }
        }
    }
    // group sums: lane (0, c) adds the partials of lanes (gg, c), gg = 1..G-1
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int q = 0; q < EPL; ++q) {
            TV t = p[r][q];
#pragma unroll
            for (int gg = 1; gg < G; ++gg) t += __shfl(p[r][q], c + gg * CPR, 64);
            p[r][q] = t;
        }
    if (lane < CPR)
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int q = 0; q < EPL; ++q) y[r * sy + (int64_t)K * B + c * EPL + q] = xo[r][q] + p[r][q];
}

template <int NP, class TM, class TV>
__global__ void __launch_bounds__(64) k_ahat_tr(int Ne, const int4* __restrict__ tb4, const TM* __restrict__ Ah,
                                                const TV* __restrict__ x, TV* __restrict__ y,
                                                const int* __restrict__ skip, const TM* const* __restrict__ Ahp = nullptr)
{
    if (skip && *skip) return;
    if (Ahp) Ah = *Ahp;
    ahat_tr_body<NP, TM, TV, 1>(blockIdx.x, tb4, Ah, x, 0, y, 0);
}

// ------------------------------------------------------------------ several right-hand sides
// R systems sharing the stored operator (x_r = x + r sx, y_r = y + r sy):
// the three blocks of the row are read from HBM once into registers and
// applied to every x_r.  The launch returns at once when every system's
// GMRES state (optional) is done.
__device__ __forceinline__ bool all_done(const GmState* __restrict__ st, int R)
{
    if (!st) return false;
    bool all = true;
    for (int r = 0; r < R; ++r) all = all && st[r].done;
    return all;
}
template <int NP, int RT>
__global__ void __launch_bounds__(64) k_ahat_fwd_m(int Ne, const int4* __restrict__ nb4, const double* __restrict__ Ah,
                                                   const double* __restrict__ x, int64_t sx, double* __restrict__ y,
                                                   int64_t sy, const GmState* __restrict__ st,
                                                   const double* const* __restrict__ Ahp = nullptr)
{
    constexpr int R = RT;
    constexpr int B = 4 * NP, BB = B * B, EPL = 2;
    constexpr int Q = fwd_chunks_per_task<B, EPL>(), EPT = Q * EPL;   // tasks as in k_ahat_fwd
    constexpr int H = BB / EPT, TPR = B / EPT, PER = (H + 63) / 64;
    __shared__ double sp[3][TPR][B + 1];
    __shared__ double sxr[R][3][B];
    if (st) {
        bool all = true;
        for (int r = 0; r < R; ++r) all = all && st[r].done;
        if (all) return;
    }
    if (Ahp) Ah = *Ahp;
    const int K = blockIdx.x, lane = threadIdx.x;
    const int4 t4 = nb4[K];
    int nbs[3];
    const uint4* src[3];
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        nbs[f] = (t4.w >> f) & 1 ? (f == 0 ? t4.x : f == 1 ? t4.y : t4.z) : -1;
        src[f] = nbs[f] >= 0 ? reinterpret_cast<const uint4*>(Ah + ((int64_t)K * 3 + f) * BB) : nullptr;
    }
    uint4 v[3][PER][Q];
#pragma unroll
    for (int f = 0; f < 3; ++f)
#pragma unroll
        for (int rr = 0; rr < PER; ++rr) {
            const int t = lane + 64 * rr;
            if (src[f] && t < H)
#pragma unroll
                for (int q = 0; q < Q; ++q) v[f][rr][q] = src[f][t * Q + q];
        }
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int f = 0; f < 3; ++f)
            if (nbs[f] >= 0 && lane < B) sxr[r][f][lane] = x[r * sx + (int64_t)nbs[f] * B + lane];
    __syncthreads();
    for (int r = 0; r < R; ++r) {
#pragma unroll
        for (int f = 0; f < 3; ++f)
#pragma unroll
            for (int rr = 0; rr < PER; ++rr) {
                const int t = lane + 64 * rr;
                if (src[f] && t < H) {
                    const int i = t / TPR, c = t % TPR;
                    double p = 0.0;
#pragma unroll
                    for (int q = 0; q < Q; ++q) {
                        const double* e = reinterpret_cast<const double*>(&v[f][rr][q]);
                        p += e[0] * sxr[r][f][c * EPT + q * EPL] + e[1] * sxr[r][f][c * EPT + q * EPL + 1];
                    }
                    sp[f][c][i] = p;
                }
            }
        __syncthreads();
        if (lane < B) {
            double acc = x[r * sx + (int64_t)K * B + lane];
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                if (nbs[f] < 0) continue;
#pragma unroll
                for (int c = 0; c < TPR; ++c) acc += sp[f][c][lane];
            }
            y[r * sy + (int64_t)K * B + lane] = acc;
        }
        __syncthreads();
    }
}

template <int NP, int R>
__global__ void __launch_bounds__(64) k_ahat_tr_m(int Ne, const int4* __restrict__ tb4, const double* __restrict__ Ah,
                                                  const double* __restrict__ x, int64_t sx, double* __restrict__ y,
                                                  int64_t sy, const GmState* __restrict__ st,
                                                  const double* const* __restrict__ Ahp = nullptr)
{
    if (all_done(st, R)) return;
    if (Ahp) Ah = *Ahp;
    ahat_tr_body<NP, double, double, R>(blockIdx.x, tb4, Ah, x, sx, y, sy);
}

// *slot = p: the operator address that captured apply launches read
__global__ void k_set_ptr(const double** __restrict__ slot, const double* p)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) *slot = p;
}

// z = a * x (FP64 -> FP32), y += a * x (FP32 -> FP64)
__global__ void k_scale_to_f32(double a, const double* __restrict__ x, float* __restrict__ z, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) z[i] = (float)(a * x[i]);
}


// out = alpha M x + beta y  (M applied block-wise)
template <int NP>
__global__ void k_mass_axpy(int Ne, const double* __restrict__ area, const double* __restrict__ mh,
                            const double* __restrict__ x, const double* __restrict__ y, double alpha, double beta,
                            double* __restrict__ out)
{
    constexpr int B = 4 * NP;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)Ne * B) return;
    int K = (int)(i / B), l = (int)(i % B), a = l >> 2, m = l & 3;
    const double* xK = x + (int64_t)K * B;
    double s = 0.0;
    for (int b = 0; b < NP; ++b) s += mh[a * NP + b] * xK[b * 4 + m];
    out[i] = alpha * 2.0 * area[K] * s + beta * y[i];
}

}  // namespace pa
