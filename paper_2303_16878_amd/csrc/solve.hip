// FP64 solve and update kernels: gauge fix and Levenberg-Marquardt damping, blocked
// Cholesky factorisation of the dense 6N x 6N system, the two triangular solves, the
// pose update X <- X exp(dx) (Supplementary: exp(dx) = [R(dq), dt], R(dq) the rotation
// of the unit quaternion with imaginary part dq) and the device-side accept/reject of a
// step, so that a whole iteration runs without returning to the host.

#include "pba_internal.h"

#include <algorithm>

namespace pba {

constexpr int NB = 64;   // Cholesky block size

// A = gauge-fixed H with Marquardt damping, rhs = -b (anchor rows zero).
// lam_override >= 0 replaces the device-side lambda (direct solve calls).
__global__ void damp_copy_kernel(const double *__restrict__ H, const double *__restrict__ b,
                                 double *__restrict__ A, double *__restrict__ rhs, int n, int anchor,
                                 const LmState *lm, double lam_override)
{
    const double lam = lam_override >= 0.0 ? lam_override : lm->lam;
    const int a0 = 6 * anchor, a1 = a0 + 6;
    const int64_t nn = (int64_t)n * n;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nn; e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / n), j = (int)(e - (int64_t)i * n);
        const bool ai = i >= a0 && i < a1, aj = j >= a0 && j < a1;
        double v = H[e];
        if (ai || aj) v = (i == j) ? 1.0 : 0.0;
        if (i == j) v += lam * v;
        A[e] = v;
        if (j == 0) rhs[i] = ai ? 0.0 : -b[i];
    }
}

void launch_damp_copy(const double *H, const double *b, double *A, double *rhs, int n, int anchor,
                      const LmState *lm, double lam_override, hipStream_t st)
{
    int64_t nn = (int64_t)n * n;
    int64_t blocks = (nn + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(damp_copy_kernel, dim3((unsigned)blocks), dim3(256), 0, st, H, b, A, rhs, n, anchor, lm,
                       lam_override);
}

// ---- blocked right-looking Cholesky, lower triangle, A row-major n x n.
// Per 64-wide block column: factor the diagonal block and invert its factor (one wave),
// form the panel below as X = B W^T with W = L_kk^-1 (tiled product), then update the
// trailing lower triangle.  The inverted diagonal blocks are kept for the solves.

// The value of v in lane l (wave-uniform l), to every lane.
__device__ __forceinline__ double bcast_lane(double v, int l)
{
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                            __builtin_amdgcn_readlane(__double2loint(v), l));
}

// 1/sqrt(d) in FP64 to about an ulp: the hardware estimate refined by two Newton steps.
__device__ __forceinline__ double rsqrt_f64(double d)
{
    double y = __builtin_amdgcn_rsq(d);
    y = y * fma(-0.5 * d * y, y, 1.5);
    return y * fma(-0.5 * d * y, y, 1.5);
}

// Factor the diagonal block at k0 and write L_kk (lower) to A and W = L_kk^-1 (lower, row-major
// 64 x 64, zero above the diagonal) to Winv.  One workgroup of 256 threads; a ragged last block is
// padded with the identity, whose factor and inverse are the identity.
//
// Right-looking over single pivots, factor and inverse together, in registers: lane i of wave w
// holds row i, columns 16 w .. 16 w + 15, of the working copy S and of V, the working rows of the
// inverse (V = I initially).  At pivot k, with p = S(k, k), c_i = S(i, k) for i > k and 0
// otherwise, and r_j = V(k, j) (zero for j > k, r_k = 1: V stays lower triangular), every element
// takes both
//   S(i, j) -= c_i c_j / p,      V(i, j) -= c_i r_j / p
// (c_j = 0 leaves S left of the pivot alone, r_j = 0 leaves V right of it alone), because
// L(i, k) = c_i / sqrt(p) and row k of the inverse is V(k, :) / sqrt(p).  Column k of S is final
// from then on, so S ends up holding L column-scaled by sqrt(p_j), and V holds W row-scaled by
// sqrt(p_i).
//
// Pivots go four at a time per barrier: the wave owning columns k .. k + 3 factors that 64 x 4
// panel on copies (cross-lane values by readlane) and publishes the four columns c as they stand
// at their pivots, with their pivots; then every wave applies the four rank-one steps in order.
// Row k + m of V, needed as r by the m-th step, is read from lane k + m of the same wave, which
// has already applied the steps before it.  No step branches on the lane or the wave.
__global__ void __launch_bounds__(256) chol_diag_kernel(double *A, int n, int k0, double *Winv, int32_t *fail)
{
    __shared__ double cb[2][4][NB];   // the four columns c of a pivot group
    __shared__ double pb[2][4];       // their pivots
    __shared__ double piv[NB];
    if (*fail) return;
    const int nb = min(NB, n - k0);
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int c0 = 16 * w;
    double a[16], v[16];
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) {
        const int j = c0 + jj;
        a[jj] = (lane < nb && j < nb) ? A[(int64_t)(k0 + lane) * n + k0 + j] : (lane == j ? 1.0 : 0.0);
        v[jj] = lane == j ? 1.0 : 0.0;
    }
    bool bad = false;
#pragma unroll 1
    for (int wo = 0; wo < 4; ++wo) {
#pragma unroll
        for (int tb = 0; tb < 4; ++tb) {
            const int kb = 4 * tb, k = 16 * wo + kb, b = tb & 1;
            if (w == wo) {
                // the 64 x 4 panel at its pivots, on copies
                double t[4] = {a[kb], a[kb + 1], a[kb + 2], a[kb + 3]};
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const double p = bcast_lane(t[m], k + m);
                    double q = __builtin_amdgcn_rcp(p);
                    q = fma(q, fma(-p, q, 1.0), q);
                    q = fma(q, fma(-p, q, 1.0), q);
                    const double c = lane > k + m ? t[m] : 0.0;
                    cb[b][m][lane] = c;
                    if (lane == 0) pb[b][m] = p;
#pragma unroll
                    for (int m2 = m + 1; m2 < 4; ++m2) t[m2] = fma(-c * q, bcast_lane(t[m], k + m2), t[m2]);
                }
            }
            __syncthreads();
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const double p = pb[b][m];
                const bool ok = p > 0.0;
                bad = bad || !ok;
                double q = __builtin_amdgcn_rcp(p);
                q = fma(q, fma(-p, q, 1.0), q);
                q = fma(q, fma(-p, q, 1.0), q);
                if (threadIdx.x == 0) piv[k + m] = ok ? p : 1.0;
                const double cr = ok ? -cb[b][m][lane] * q : 0.0;
#pragma unroll
                for (int jj = 0; jj < 16; ++jj) {
                    a[jj] = fma(cr, cb[b][m][c0 + jj], a[jj]);
                    v[jj] = fma(cr, bcast_lane(v[jj], k + m), v[jj]);
                }
            }
        }
    }
    __syncthreads();
    double *Wb = Winv + (int64_t)(k0 / NB) * NB * NB;
    const double si = rsqrt_f64(piv[lane]);
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) {
        const int j = c0 + jj;
        const bool low = j <= lane, in = lane < nb && j < nb;
        Wb[lane * NB + j] = (low && in) ? v[jj] * si : 0.0;
        if (low && in) A[(int64_t)(k0 + lane) * n + k0 + j] = a[jj] * rsqrt_f64(piv[j]);
    }
    if (threadIdx.x == 0 && bad) *fail = 1;
}

// Panel below the diagonal block: X = B W^T for 64 rows per workgroup (16 x 16 threads, 4 x 4 each).
__global__ void __launch_bounds__(256) chol_trsm_kernel(double *A, int n, int k0, const double *Winv,
                                                        const int32_t *__restrict__ tiles, const int32_t *fail)
{
    __shared__ double Bs[NB][NB + 1];
    __shared__ double Ws[NB][NB + 1];
    if (*fail) return;
    const int nb = min(NB, n - k0);
    const int r0 = tiles[blockIdx.x] * NB;   // a tile row below the diagonal block
    const int rows = min(NB, n - r0);
    const int tid = threadIdx.x;
    const double *Wb = Winv + (int64_t)(k0 / NB) * NB * NB;
    for (int e = tid; e < NB * NB; e += blockDim.x) {
        const int i = e / NB, k = e % NB;
        Bs[i][k] = (i < rows && k < nb) ? A[(int64_t)(r0 + i) * n + k0 + k] : 0.0;
        Ws[i][k] = Wb[e];
    }
    __syncthreads();
    const int tx = tid & 15, ty = tid >> 4;
    double c[4][4];
    for (int a = 0; a < 4; ++a)
        for (int q = 0; q < 4; ++q) c[a][q] = 0.0;
    for (int k = 0; k < nb; ++k) {
        double b[4], w[4];
        for (int a = 0; a < 4; ++a) b[a] = Bs[ty * 4 + a][k];
        for (int q = 0; q < 4; ++q) w[q] = Ws[tx * 4 + q][k];
        for (int a = 0; a < 4; ++a)
            for (int q = 0; q < 4; ++q) c[a][q] += b[a] * w[q];
    }
    for (int a = 0; a < 4; ++a)
        for (int q = 0; q < 4; ++q) {
            const int i = ty * 4 + a, j = tx * 4 + q;
            if (i < rows && j < nb) A[(int64_t)(r0 + i) * n + k0 + j] = c[a][q];
        }
}

// Trailing update A_ij -= L_i L_j^T for block pairs i >= j below the panel.
__global__ void __launch_bounds__(256) chol_update_kernel(double *A, int n, int k0, const int32_t *__restrict__ tiles,
                                                          const int32_t *fail)
{
    __shared__ double Li[NB][NB + 1];
    __shared__ double Lj[NB][NB + 1];
    if (*fail) return;
    const int nb = min(NB, n - k0);
    // blockIdx.x -> (bi, bj) with bi >= bj over the panel's tile rows
    const int idx = blockIdx.x;
    int bi = (int)((sqrt(8.0 * idx + 1.0) - 1.0) * 0.5);
    while ((bi + 1) * (bi + 2) / 2 <= idx) ++bi;
    while (bi * (bi + 1) / 2 > idx) --bi;
    const int bj = idx - bi * (bi + 1) / 2;
    const int ri = tiles[bi] * NB, rj = tiles[bj] * NB;
    const int ni = min(NB, n - ri), nj = min(NB, n - rj);
    const int tid = threadIdx.x;
    for (int e = tid; e < NB * NB; e += blockDim.x) {
        const int i = e / NB, k = e % NB;
        Li[i][k] = (i < ni && k < nb) ? A[(int64_t)(ri + i) * n + k0 + k] : 0.0;
        Lj[i][k] = (i < nj && k < nb) ? A[(int64_t)(rj + i) * n + k0 + k] : 0.0;
    }
    __syncthreads();
    const int tx = tid & 15, ty = tid >> 4;
    double c[4][4];
    for (int a = 0; a < 4; ++a)
        for (int q = 0; q < 4; ++q) c[a][q] = 0.0;
    for (int k = 0; k < nb; ++k) {
        double li[4], lj[4];
        for (int a = 0; a < 4; ++a) li[a] = Li[ty * 4 + a][k];
        for (int q = 0; q < 4; ++q) lj[q] = Lj[tx * 4 + q][k];
        for (int a = 0; a < 4; ++a)
            for (int q = 0; q < 4; ++q) c[a][q] += li[a] * lj[q];
    }
    for (int a = 0; a < 4; ++a)
        for (int q = 0; q < 4; ++q) {
            const int i = ty * 4 + a, j = tx * 4 + q;
            if (i < ni && j < nj && (bi != bj || j <= i)) A[(int64_t)(ri + i) * n + rj + j] -= c[a][q];
        }
}

__global__ void reset_flag_kernel(int32_t *f) { *f = 0; }

void launch_cholesky(double *A, int n, double *Winv, const CholPlan &plan, int32_t *fail, hipStream_t st)
{
    hipLaunchKernelGGL(reset_flag_kernel, dim3(1), dim3(1), 0, st, fail);
    const int nblk = (n + NB - 1) / NB;
    for (int kb = 0; kb < nblk; ++kb) {
        const int k0 = kb * NB;
        hipLaunchKernelGGL(chol_diag_kernel, dim3(1), dim3(256), 0, st, A, n, k0, Winv, fail);
        const int m = plan.rcnt[kb];
        if (m > 0) {
            const int32_t *tiles = plan.rows + plan.rbeg[kb];
            hipLaunchKernelGGL(chol_trsm_kernel, dim3(m), dim3(256), 0, st, A, n, k0, Winv, tiles, fail);
            hipLaunchKernelGGL(chol_update_kernel, dim3(m * (m + 1) / 2), dim3(256), 0, st, A, n, k0, tiles, fail);
        }
    }
}

// L y = rhs, then L^T x = y, as one launch per 64-row block and direction (right-looking, so each
// launch spreads over many workgroups).  The right-hand side in x is consumed; y lives in the n
// doubles of workspace that follow the inverted diagonal blocks in Winv; x receives the solution
// (zero if the factorisation failed).

// Forward block kb: y_k = W_kk r_k, then r_i -= L_ik y_k for the rows below.  Workgroup g owns
// the 64 rows of the g-th tile row in the block column's list; every workgroup forms y_k itself
// (r_k is not written in this launch), workgroup 0 stores it.
__global__ void __launch_bounds__(256) trsv_fwd_kernel(const double *__restrict__ L, const double *__restrict__ Winv,
                                                       double *__restrict__ r, double *__restrict__ y, int n, int kb,
                                                       const int32_t *__restrict__ tiles, int ntiles,
                                                       const int32_t *fail)
{
    __shared__ double sy[NB];
    if (*fail) return;
    const int k0 = kb * NB, nb = min(NB, n - k0);
    const int tid = threadIdx.x, row = tid >> 2, part = tid & 3;
    const double *Wb = Winv + (int64_t)kb * NB * NB;
    double s = 0.0;
#pragma unroll
    for (int c = part * 16; c < part * 16 + 16; ++c) s += c < nb ? Wb[row * NB + c] * r[k0 + c] : 0.0;
    s += __shfl_xor(s, 1, 64);
    s += __shfl_xor(s, 2, 64);
    if (part == 0) sy[row] = s;
    __syncthreads();
    if (blockIdx.x == 0 && tid < nb) y[k0 + tid] = sy[tid];
    // the tile row this workgroup updates (none when block kb couples to no row below it)
    const int i = (ntiles > 0 ? tiles[blockIdx.x] * NB : n) + row;
    double u = 0.0;
    if (i < n) {
        const double *Lr = L + (int64_t)i * n + k0;
#pragma unroll
        for (int c = part * 16; c < part * 16 + 16; ++c) u += c < nb ? Lr[c] * sy[c] : 0.0;
    }
    u += __shfl_xor(u, 1, 64);
    u += __shfl_xor(u, 2, 64);
    if (i < n && part == 0) r[i] -= u;
}

// Backward block kb: x_k = W_kk^T s_k, then s_i -= sum_c L[k0 + c][i] x_k[c] for the columns
// i < k0.  Workgroup g owns the 64 columns of the g-th tile in the block row's list; workgroup 0
// stores x_k.
__global__ void __launch_bounds__(256) trsv_bwd_kernel(const double *__restrict__ L, const double *__restrict__ Winv,
                                                       double *__restrict__ s, double *__restrict__ x, int n, int kb,
                                                       const int32_t *__restrict__ tiles, int ntiles,
                                                       const int32_t *fail)
{
    __shared__ double sx[NB];
    __shared__ double part_s[4][NB];
    if (*fail) return;
    const int k0 = kb * NB, nb = min(NB, n - k0);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const double *Wb = Winv + (int64_t)kb * NB * NB;
    {
        // x_k[c] = sum_i W[i][c] s_k[i]: wave wv sums rows 16 wv .. 16 wv + 15 for column `lane`
        double t = 0.0;
#pragma unroll
        for (int i = wv * 16; i < wv * 16 + 16; ++i) t += i < nb ? Wb[i * NB + lane] * s[k0 + i] : 0.0;
        part_s[wv][lane] = t;
    }
    __syncthreads();
    if (tid < NB) sx[tid] = part_s[0][tid] + part_s[1][tid] + part_s[2][tid] + part_s[3][tid];
    __syncthreads();
    if (blockIdx.x == 0 && tid < nb) x[k0 + tid] = sx[tid];
    // the tile column this workgroup updates (none when block row kb couples to no column left of it)
    const int i = (ntiles > 0 ? tiles[blockIdx.x] * NB : k0) + lane;
    double u = 0.0;
    if (i < k0) {
#pragma unroll
        for (int c = wv * 16; c < wv * 16 + 16; ++c) u += c < nb ? L[(int64_t)(k0 + c) * n + i] * sx[c] : 0.0;
    }
    __syncthreads();
    part_s[wv][lane] = u;
    __syncthreads();
    if (wv == 0 && i < k0) s[i] -= part_s[0][lane] + part_s[1][lane] + part_s[2][lane] + part_s[3][lane];
}

__global__ void zero_on_fail_kernel(double *x, int n, const int32_t *fail)
{
    if (!*fail) return;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) x[i] = 0.0;
}

void launch_chol_solve(const double *L, double *Winv, double *x, int n, const CholPlan &plan, const int32_t *fail,
                       hipStream_t st)
{
    const int nblk = (n + NB - 1) / NB;
    double *y = Winv + (int64_t)nblk * NB * NB;
    for (int kb = 0; kb < nblk; ++kb) {
        const int m = plan.rcnt[kb];
        hipLaunchKernelGGL(trsv_fwd_kernel, dim3(std::max(m, 1)), dim3(256), 0, st, L, Winv, x, y, n, kb,
                           plan.rows + plan.rbeg[kb], m, fail);
    }
    for (int kb = nblk - 1; kb >= 0; --kb) {
        const int m = plan.ccnt[kb];
        hipLaunchKernelGGL(trsv_bwd_kernel, dim3(std::max(m, 1)), dim3(256), 0, st, L, Winv, y, x, n, kb,
                           plan.cols + plan.cbeg[kb], m, fail);
    }
    hipLaunchKernelGGL(zero_on_fail_kernel, dim3((n + 255) / 256), dim3(256), 0, st, x, n, fail);
}

// ---- pose update

__device__ static void quat_rot(double qx, double qy, double qz, double *R)
{
    double n2 = qx * qx + qy * qy + qz * qz, w;
    if (n2 < 1.0) {
        w = sqrt(1.0 - n2);
    } else {
        const double s = 1.0 / sqrt(1.0 + n2);
        w = s; qx *= s; qy *= s; qz *= s;
    }
    R[0] = 1 - 2 * (qy * qy + qz * qz); R[1] = 2 * (qx * qy - qz * w);     R[2] = 2 * (qx * qz + qy * w);
    R[3] = 2 * (qx * qy + qz * w);     R[4] = 1 - 2 * (qx * qx + qz * qz); R[5] = 2 * (qy * qz - qx * w);
    R[6] = 2 * (qx * qz - qy * w);     R[7] = 2 * (qy * qz + qx * w);     R[8] = 1 - 2 * (qx * qx + qy * qy);
}

// Xout_k = X_k exp(dx_k); also the step norm into lm (one workgroup reduces it).
__global__ void __launch_bounds__(256) boxplus_kernel(const double *__restrict__ X, const double *__restrict__ dx,
                                                      double *__restrict__ Xo, int N, const int32_t *fail,
                                                      LmState *lm)
{
    const int tid = threadIdx.x;
    const bool f = fail && *fail;
    __shared__ double red[256];
    double ss = 0.0;
    for (int k = tid; k < N; k += blockDim.x) {
        const double *x = X + 12 * (int64_t)k;
        double *o = Xo + 12 * (int64_t)k;
        if (f) {
            for (int i = 0; i < 12; ++i) o[i] = x[i];
            continue;
        }
        const double *d = dx + 6 * (int64_t)k;
        for (int i = 0; i < 6; ++i) ss += d[i] * d[i];
        double E[9];
        quat_rot(d[3], d[4], d[5], E);
        double R[9];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) R[3 * i + j] = x[3 * i] * E[j] + x[3 * i + 1] * E[3 + j] + x[3 * i + 2] * E[6 + j];
        for (int i = 0; i < 3; ++i) o[9 + i] = x[9 + i] + x[3 * i] * d[0] + x[3 * i + 1] * d[1] + x[3 * i + 2] * d[2];
        for (int i = 0; i < 9; ++i) o[i] = R[i];
    }
    red[tid] = ss;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    if (tid == 0 && lm) {
        lm->step_norm = sqrt(red[0]);
        lm->fail = f ? 1 : 0;
    }
}

void launch_boxplus(const double *X, const double *dx, double *Xout, int N, const int32_t *fail, LmState *lm,
                    hipStream_t st)
{
    hipLaunchKernelGGL(boxplus_kernel, dim3(1), dim3(256), 0, st, X, dx, Xout, N, fail, lm);
}

// Accept/reject the candidate: totals_cand = {F, evaluated, valid, 0} at the candidate
// poses.  Gauss-Newton (use_lm = 0) accepts every solved step; LM accepts if F decreases.
// On accept the candidate system, gradient and poses become current.  Writes one log row
// {F, lambda, step_norm, valid, accepted}.
__global__ void __launch_bounds__(256) lm_decide_kernel(LmState *lm, const double *__restrict__ totals_cand,
                                                        int64_t nH, double *H_cur, const double *H_cand,
                                                        double *b_cur, const double *b_cand, int nb,
                                                        double *X_cur, const double *X_cand, int nX)
{
    __shared__ int acc;
    const double Fc = totals_cand[0];
    const bool solved = !lm->fail;
    const bool accept = solved && (!lm->use_lm || Fc < lm->F_cur);
    if (threadIdx.x == 0) acc = accept;
    __syncthreads();
    if (acc) {
        const int64_t stride = (int64_t)gridDim.x * blockDim.x;
        for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nH; e += stride) H_cur[e] = H_cand[e];
        for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nb; e += stride) b_cur[e] = b_cand[e];
        for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nX; e += stride) X_cur[e] = X_cand[e];
    }
}

// Scalar part of the decision, run after the copies (single thread).
__global__ void lm_finish_kernel(LmState *lm, const double *__restrict__ totals_cand, double *totals_cur,
                                 double *logbuf, int log_cap)
{
    // the row is chosen on the device so that every iteration launches identical arguments
    double *log_row = logbuf + 8 * (int64_t)min(lm->iter, log_cap - 1);
    const double Fc = totals_cand[0];
    const bool solved = !lm->fail;
    const bool accept = solved && (!lm->use_lm || Fc < lm->F_cur);
    if (accept) {
        for (int k = 0; k < 4; ++k) totals_cur[k] = totals_cand[k];
        lm->F_cur = Fc;
        lm->valid_cur = (int64_t)totals_cand[2];
        if (lm->use_lm) lm->lam = fmax(lm->lam / 10.0, 1e-12);
    } else if (lm->use_lm) {
        lm->lam *= 10.0;
    }
    lm->accepted = accept;
    log_row[0] = lm->F_cur;
    log_row[1] = lm->use_lm ? lm->lam : 0.0;
    log_row[2] = solved ? lm->step_norm : 0.0;
    log_row[3] = (double)lm->valid_cur;
    log_row[4] = accept ? 1.0 : 0.0;
    log_row[5] = solved ? 0.0 : 1.0;
    lm->iter += 1;
}

void launch_lm_decide(LmState *lm, const double *totals_cand, int64_t nH, double *H_cur, const double *H_cand,
                      double *b_cur, const double *b_cand, double *X_cur, const double *X_cand, int N,
                      double *totals_cur, double *logbuf, int log_cap, hipStream_t st)
{
    int64_t blocks = (nH + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(lm_decide_kernel, dim3((unsigned)blocks), dim3(256), 0, st, lm, totals_cand, nH, H_cur, H_cand,
                       b_cur, b_cand, 6 * N, X_cur, X_cand, 12 * N);
    hipLaunchKernelGGL(lm_finish_kernel, dim3(1), dim3(1), 0, st, lm, totals_cand, totals_cur, logbuf, log_cap);
}

__global__ void copy_kernel(double *__restrict__ dst, const double *__restrict__ src, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// Device wall-clock stamp (constant-rate counter) into slot 6 + which of the current iteration's
// log row: the evaluation inside a captured iteration is bracketed by two of these, so every
// replay of the graph leaves its own evaluation duration.
__global__ void stamp_kernel(const LmState *lm, double *logbuf, int log_cap, int which)
{
    if (threadIdx.x != 0) return;
    uint64_t *row = reinterpret_cast<uint64_t *>(logbuf + 8 * (int64_t)min(lm->iter, log_cap - 1));
    row[6 + which] = (uint64_t)wall_clock64();
}

void launch_stamp(const LmState *lm, double *logbuf, int log_cap, int which, hipStream_t st)
{
    hipLaunchKernelGGL(stamp_kernel, dim3(1), dim3(64), 0, st, lm, logbuf, log_cap, which);
}

void launch_copy(double *dst, const double *src, int64_t n, hipStream_t st)
{
    if (n <= 0) return;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(copy_kernel, dim3((unsigned)blocks), dim3(256), 0, st, dst, src, n);
}

}  // namespace pba
