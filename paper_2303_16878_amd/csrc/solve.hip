// FP64 solve and update kernels: gauge fix and Levenberg-Marquardt damping, blocked
// Cholesky factorisation of the dense 6N x 6N system, the two triangular solves, the
// pose update X <- X exp(dx) (Supplementary: exp(dx) = [R(dq), dt], R(dq) the rotation
// of the unit quaternion with imaginary part dq) and the device-side accept/reject of a
// step, so that a whole iteration runs without returning to the host.

#include "pba_internal.h"

#include <algorithm>
#include <cstdlib>

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

// The same system in a nested-dissection order: factor row R holds row perm[R] of the 6 NP system
// (perm[R] < 0: padding, a unit diagonal and no coupling).  Only the lower tiles of the factor's
// pattern are written (one workgroup per tile, dtiles), the diagonal tiles in full; rhs is the
// permuted -b.  Also clears the failure flag ahead of the level launches.
__global__ void __launch_bounds__(256) damp_copy_perm_kernel(const double *__restrict__ H,
                                                             const double *__restrict__ b, double *__restrict__ A,
                                                             double *__restrict__ rhs, int n0, int n,
                                                             const int32_t *__restrict__ perm,
                                                             const int32_t *__restrict__ dtiles, int anchor,
                                                             const LmState *lm, double lam_override, int32_t *fail)
{
    const double lam = lam_override >= 0.0 ? lam_override : lm->lam;
    const int a0 = 6 * anchor, a1 = a0 + 6;
    const int ti = dtiles[2 * blockIdx.x], tj = dtiles[2 * blockIdx.x + 1];
    const int C = tj * NB + (threadIdx.x & 63), oc = perm[C];
    const bool ac = oc >= a0 && oc < a1;
    for (int r = threadIdx.x >> 6; r < NB; r += 4) {
        const int R = ti * NB + r, orow = perm[R];
        const bool ar = orow >= a0 && orow < a1;
        double v = (orow >= 0 && oc >= 0) ? H[(int64_t)orow * n0 + oc] : 0.0;
        if (orow < 0 || oc < 0 || ar || ac) v = (R == C) ? 1.0 : 0.0;
        if (R == C) v += lam * v;
        A[(int64_t)R * n + C] = v;
    }
    if (ti == tj && threadIdx.x < NB) {
        const int R = ti * NB + threadIdx.x, o = perm[R];
        rhs[R] = (o < 0 || (o >= a0 && o < a1)) ? 0.0 : -b[o];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *fail = 0;
}

void launch_damp_copy_perm(const double *H, const double *b, double *A, double *rhs, int n0, int anchor,
                           const LmState *lm, double lam_override, const CholPlan &plan, int32_t *fail, hipStream_t st)
{
    hipLaunchKernelGGL(damp_copy_perm_kernel, dim3(plan.ndt), dim3(256), 0, st, H, b, A, rhs, n0, plan.n, plan.perm,
                       plan.dtiles, anchor, lm, lam_override, fail);
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
// Per 64-wide block column: factor the diagonal block and invert its factor (one workgroup),
// then, in one launch, form the panel below as X = B W^T with W = L_kk^-1 and update the
// trailing lower triangle with it.  The panel tiles of the factor go to a second n x n matrix
// (A itself keeps the input panel, which the same launch reads); the inverted diagonal blocks
// are kept for the solves.

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

// Factor the diagonal block at k0 and write W = L_kk^-1 (lower, row-major 64 x 64, zero above the
// diagonal) and W^T to Winv (blocks k0 / 64 and nblk + k0 / 64); the factor itself is not needed
// (the panel and the solves use W).  One workgroup of 256 threads; a ragged last block is padded
// with the identity, whose factor and inverse are the identity.
//
// Right-looking over single pivots, factor and inverse together, in registers: lane i of wave w
// holds S(i, 16 w + jj), row i of the working copy S, and lane j of wave w holds V(16 w + jj, j),
// column j of the working rows of the inverse (V = I initially), jj = 0..15.  At pivot k, with
// p = S(k, k), c_i = S(i, k) for i > k and 0 otherwise, and r_j = V(k, j) (zero for j > k, r_k = 1:
// V stays lower triangular), every element takes both
//   S(i, j) -= c_i c_j / p,      V(i, j) -= c_i r_j / p
// (c_j = 0 leaves S left of the pivot alone, r_j = 0 leaves V right of it alone), because
// L(i, k) = c_i / sqrt(p) and row k of the inverse is V(k, :) / sqrt(p).  Column k of S is final
// from then on, and V ends up holding W row-scaled by sqrt(p_i).  Both updates of a wave use the
// same 16 values c_(16 w + jj), read from LDS as broadcasts, and one value per lane (c_i for S,
// r_j for V).
//
// Pivots go four at a time per barrier: the wave owning columns k .. k + 3 of S (and rows
// k .. k + 3 of V) factors that 64 x 4 panel on copies (cross-lane values by readlane), carries
// the four rows of V along, and publishes the four columns c and rows r as they stand at their
// pivots, with the pivots and their reciprocals; then every wave applies the four rank-one steps
// in order.  No step branches on the lane or the wave.  (Broadcasting the 16 values by readlane
// instead of LDS, skipping the column ranges a step cannot change, or eight pivots per barrier
// all measured slower; keeping V with lane = row, which needs 32 readlanes per pivot, cost 30%.)
//
// kList: the launch factors the block columns cols[blockIdx.x] (one tree level of a nested-dissection
// order; the failure flag was cleared before the factorisation), else the single block at k0, the
// first of which (k0 = 0) clears the flag.  With x (kList only), the forward substitution's step
// of the block rides along: x_k holds r_k, the right-hand side with every earlier column's
// contribution already subtracted (by the update launches), and becomes y_k = W r_k.
template <bool kList>
__global__ void __launch_bounds__(256) chol_diag_kernel(const double *A, int n, int k0_arg,
                                                        const int32_t *__restrict__ cols, double *Winv,
                                                        int32_t *fail, double *x)
{
    __shared__ double cb[2][4][NB];   // the four columns c of a pivot group (double-buffered)
    __shared__ double rb[2][4][NB];   // the four rows r of V at their pivots
    __shared__ double pb[2][4];       // the pivots
    __shared__ double qb[2][4];       // their reciprocals
    __shared__ double piv[NB];
    __shared__ double Ts[NB][NB + 1];   // W, transposed on the way out
    const int k0 = kList ? cols[blockIdx.x] * NB : k0_arg;
    const bool clears = !kList && k0 == 0;
    if (!clears && *fail) return;
    const int nb = min(NB, n - k0);
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int c0 = 16 * w;
    double a[16], v[16];   // S(lane, c0 + jj), V(c0 + jj, lane)
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
                double t[4], r[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    t[m] = a[kb + m];
                    r[m] = v[kb + m];
                }
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const double p = bcast_lane(t[m], k + m);
                    double q = __builtin_amdgcn_rcp(p);
                    q = fma(q, fma(-p, q, 1.0), q);
                    q = fma(q, fma(-p, q, 1.0), q);
                    const double c = lane > k + m ? t[m] : 0.0;
                    cb[b][m][lane] = c;
                    rb[b][m][lane] = r[m];
                    if (lane == 0) {
                        pb[b][m] = p;
                        qb[b][m] = q;
                    }
#pragma unroll
                    for (int m2 = m + 1; m2 < 4; ++m2) {
                        const double cm2 = bcast_lane(t[m], k + m2);
                        t[m2] = fma(-c * q, cm2, t[m2]);
                        r[m2] = fma(-cm2 * q, r[m], r[m2]);
                    }
                }
            }
            __syncthreads();
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const double p = pb[b][m];
                const bool ok = p > 0.0;
                bad = bad || !ok;
                if (threadIdx.x == 0) piv[k + m] = ok ? p : 1.0;
                const double qq = ok ? qb[b][m] : 0.0;
                const double cr = -cb[b][m][lane] * qq, rr = -rb[b][m][lane] * qq;
#pragma unroll
                for (int jj = 0; jj < 16; ++jj) {
                    const double cj = cb[b][m][c0 + jj];
                    a[jj] = fma(cr, cj, a[jj]);
                    v[jj] = fma(rr, cj, v[jj]);
                }
            }
        }
    }
    __syncthreads();
    double *Wb = Winv + (int64_t)(k0 / NB) * NB * NB;
    double *Wtb = Winv + (int64_t)((n + NB - 1) / NB + k0 / NB) * NB * NB;
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) {
        const int i = c0 + jj;
        const double sp = rsqrt_f64(piv[i]);
        const bool low = lane <= i, in = i < nb && lane < nb;
        const double wv = (low && in) ? v[jj] * sp : 0.0;
        Wb[i * NB + lane] = wv;
        Ts[lane][i] = wv;
    }
    __syncthreads();
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) Wtb[(c0 + jj) * NB + lane] = Ts[c0 + jj][lane];
    if (threadIdx.x == 0 && (bad || clears)) *fail = bad ? 1 : 0;
    if (kList && x) {   // y_k = W r_k: row i = t / 4, columns 16 (t % 4) .. +15 (Ts[j][i] = W(i, j))
        double *rk = x + k0;
        if (threadIdx.x < NB) piv[threadIdx.x] = rk[threadIdx.x];   // r_k (the pivots are no longer needed)
        __syncthreads();
        const int i = threadIdx.x >> 2, j0 = (threadIdx.x & 3) * 16;
        double y = 0.0;
#pragma unroll
        for (int j = 0; j < 16; ++j) y = fma(Ts[j0 + j][i], piv[j0 + j], y);
        y += __shfl_xor(y, 1, 64);
        y += __shfl_xor(y, 2, 64);
        if ((threadIdx.x & 3) == 0) rk[i] = y;
    }
}

// C += P Q^T over k = 0..63 for tiles in LDS (rows padded to 65 doubles), 16 x 16 threads,
// RA x RB outputs each: rows ty + 16 a of P, rows tx + 16 b of Q.  With the odd row pitch the 16
// rows a wave reads from Q fall in distinct banks (rows 4 tx + b would collide four ways).
template <int RA, int RB>
__device__ __forceinline__ void tile_nt(const double (*P)[NB + 1], const double (*Q)[NB + 1], int tx, int ty,
                                        double (&c)[RA][RB])
{
#pragma unroll 32
    for (int k = 0; k < NB; ++k) {
        double p[RA], q[RB];
#pragma unroll
        for (int a = 0; a < RA; ++a) p[a] = P[ty + 16 * a][k];
#pragma unroll
        for (int b = 0; b < RB; ++b) q[b] = Q[tx + 16 * b][k];
#pragma unroll
        for (int a = 0; a < RA; ++a)
#pragma unroll
            for (int b = 0; b < RB; ++b) c[a][b] = fma(p[a], q[b], c[a][b]);
    }
}

// Rows r0 .. r0 + R - 1 (those below `rows`), columns c0 .. c0 + nc - 1 of the row-major matrix M
// (row pitch ld, even; c0 and nc even) into a zero-padded R x 64 LDS tile, by a 256-thread
// workgroup.  All of a thread's 16-byte loads are issued before the first is used.
template <int R>
__device__ __forceinline__ void load_tile(double (*T)[NB + 1], const double *M, int64_t ld, int rows, int r0,
                                          int c0, int nc)
{
    constexpr int kIt = R * NB / 2 / 256;
    double2 v[kIt];
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
        const int e = it * 256 + (int)threadIdx.x, i = e >> 5, k = (e & 31) * 2;
        v[it] = (r0 + i < rows && k < nc) ? *reinterpret_cast<const double2 *>(M + (r0 + i) * ld + c0 + k)
                                          : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
        const int e = it * 256 + (int)threadIdx.x, i = e >> 5, k = (e & 31) * 2;
        T[i][k] = v[it].x;
        T[i][k + 1] = v[it].y;
    }
}

// Panel and trailing update of block column k0 in one launch, four workgroups per pair (bi, bj),
// bi >= bj, of the column's tile rows (ascending list `tiles`).  Workgroup (pair, qi, qj) takes
// rows 32 qi .. 32 qi + 31 of tile row bi and rows 32 qj .. 32 qj + 31 of tile row bj: it forms
// those rows of the panel, X = B W^T, from the input panel B in A, then applies A_ij -= X_i X_j^T
// to its 32 x 32 quarter of tile (bi, bj).  On the diagonal pairs the quarter above the diagonal
// has nothing to do, and the workgroups with qj = 0 write their rows of X_i to L and L^T.  Panel rows are
// recomputed by the workgroups that need them, so no workgroup waits for another.
__global__ void __launch_bounds__(256) chol_panel_update_kernel(double *A, double *L, double *LT, int n, int k0,
                                                                const double *__restrict__ Winv,
                                                                const int32_t *__restrict__ tiles,
                                                                const int32_t *fail)
{
    constexpr int H = NB / 2;
    __shared__ double Ws[NB][NB + 1];
    __shared__ double Xi[H][NB + 1];
    __shared__ double Xj[H][NB + 1];
    if (*fail) return;
    const int nb = min(NB, n - k0);
    const int idx = blockIdx.x >> 2, qi = (blockIdx.x >> 1) & 1, qj = blockIdx.x & 1;
    int bi = (int)((sqrt(8.0 * idx + 1.0) - 1.0) * 0.5);
    while ((bi + 1) * (bi + 2) / 2 <= idx) ++bi;
    while (bi * (bi + 1) / 2 > idx) --bi;
    const int bj = idx - bi * (bi + 1) / 2;
    const bool diag = bi == bj;
    const int ri = tiles[bi] * NB + H * qi, rj = tiles[bj] * NB + H * qj;
    const int ni = min(H, n - ri), nj = min(H, n - rj);
    if ((diag && qj > qi) || ni <= 0 || nj <= 0) return;   // uniform over the workgroup
    const bool same = diag && qi == qj;                      // X_j rows are X_i's
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    load_tile<NB>(Ws, Winv + (int64_t)(k0 / NB) * NB * NB, NB, NB, 0, 0, NB);
    load_tile<H>(Xi, A, n, n, ri, k0, nb);
    if (!same) load_tile<H>(Xj, A, n, n, rj, k0, nb);
    __syncthreads();
    // X = B W^T in place: the results stay in registers until every thread has read B
    double ci[2][4] = {}, cj[2][4] = {};
    tile_nt(Xi, Ws, tx, ty, ci);
    if (!same) tile_nt(Xj, Ws, tx, ty, cj);
    __syncthreads();
    const bool write_l = diag && qj == 0;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = ty + 16 * a, j = tx + 16 * q;
            Xi[i][j] = ci[a][q];
            if (!same) Xj[i][j] = cj[a][q];
            if (write_l && i < ni && j < nb) L[(int64_t)(ri + i) * n + k0 + j] = ci[a][q];
        }
    __syncthreads();
    if (write_l)   // the same rows into L^T, read back column-wise so the stores run along its rows
        for (int e = tid; e < H * NB; e += 256) {
            const int i = e % H, j = e / H;
            if (i < ni && j < nb) LT[(int64_t)(k0 + j) * n + ri + i] = Xi[i][j];
        }
    double c[2][2] = {};
    tile_nt(Xi, same ? Xi : Xj, tx, ty, c);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int i = ty + 16 * a, j = tx + 16 * q;
            if (i < ni && j < nj && (!diag || H * qj + j <= H * qi + i)) A[(int64_t)(ri + i) * n + rj + j] -= c[a][q];
        }
}

// One elimination-tree level of a nested-dissection factorisation, after its diagonal blocks: every
// block column k of the level contributes A_ab -= X_a X_b^T, X = A_(., k) W_k^T, to the tiles (a, b),
// b <= a, of its tile rows, and writes X as its panel of the factor.  The tiles a level writes
// belong to higher levels, so no tile is both read as a panel and updated here.  One task per
// target tile lists its contributing columns (ascending); workgroup (task, qi, qj) owns one
// 32 x 32 quarter of the target and sums the contributions in registers, column by column in
// that order, before subtracting them: the result does not depend on the schedule.  The
// workgroups of a diagonal target with qj = 0 write their rows of each contributor's panel to L
// and L^T.
//
// The forward substitution rides along: the diagonal targets' workgroups, which form each
// contributor's panel rows X_a = L_ak anyway, subtract L_ak y_k from their rows r_a of x (y_k was
// written by this level's diagonal launch; r_a belongs to a higher level and only this task
// writes it).
__global__ void __launch_bounds__(256) chol_level_update_kernel(double *A, double *L, double *LT, int n,
                                                                const double *__restrict__ Winv,
                                                                const int32_t *__restrict__ tasks,
                                                                const int32_t *__restrict__ contrib,
                                                                const int32_t *fail, double *x)
{
    constexpr int H = NB / 2;
    __shared__ double Ws[NB][NB + 1];
    __shared__ double Xi[H][NB + 1];
    __shared__ double Xj[H][NB + 1];
    if (*fail) return;
    const int4 tk = reinterpret_cast<const int4 *>(tasks)[blockIdx.x >> 2];
    const int qi = (blockIdx.x >> 1) & 1, qj = blockIdx.x & 1;
    const bool diag = tk.x == tk.y;
    if (diag && qj > qi) return;   // uniform over the workgroup
    const bool same = diag && qi == qj, write_l = diag && qj == 0;
    const int ri = tk.x * NB + H * qi, rj = tk.y * NB + H * qj;
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    double c[2][2] = {};
    double z = 0.0;   // write_l: sum over the contributors of L_ak y_k, row tid / 8 of the quarter
    for (int e = 0; e < tk.w; ++e) {
        const int kb = contrib[tk.z + e], k0 = kb * NB;
        load_tile<NB>(Ws, Winv + (int64_t)kb * NB * NB, NB, NB, 0, 0, NB);
        load_tile<H>(Xi, A, n, n, ri, k0, NB);
        if (!same) load_tile<H>(Xj, A, n, n, rj, k0, NB);
        __syncthreads();
        double ci[2][4] = {}, cj[2][4] = {};
        tile_nt(Xi, Ws, tx, ty, ci);
        if (!same) tile_nt(Xj, Ws, tx, ty, cj);
        __syncthreads();
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = ty + 16 * a, j = tx + 16 * q;
                Xi[i][j] = ci[a][q];
                if (!same) Xj[i][j] = cj[a][q];
                if (write_l) L[(int64_t)(ri + i) * n + k0 + j] = ci[a][q];
            }
        __syncthreads();
        if (write_l) {
            for (int e2 = tid; e2 < H * NB; e2 += 256) {
                const int i = e2 % H, j = e2 / H;
                LT[(int64_t)(k0 + j) * n + ri + i] = Xi[i][j];
            }
            const int i = tid >> 3, j0 = (tid & 7) * 8;   // 8 lanes per row, 8 columns each
#pragma unroll
            for (int j = 0; j < 8; ++j) z = fma(Xi[i][j0 + j], x[k0 + j0 + j], z);
        }
        tile_nt(Xi, same ? Xi : Xj, tx, ty, c);
        __syncthreads();   // the next contributor's tiles overwrite the LDS
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int i = ty + 16 * a, j = tx + 16 * q;
            if (!diag || H * qj + j <= H * qi + i) A[(int64_t)(ri + i) * n + rj + j] -= c[a][q];
        }
    if (write_l && x) {   // uniform over the workgroup
        z += __shfl_xor(z, 1, 64);
        z += __shfl_xor(z, 2, 64);
        z += __shfl_xor(z, 4, 64);
        if ((tid & 7) == 0) x[ri + (tid >> 3)] -= z;
    }
}

void launch_cholesky(double *A, double *L, double *LT, int n, double *Winv, const CholPlan &plan, int32_t *fail,
                     hipStream_t st, double *x)
{
    if (plan.nd) {
        for (size_t l = 0; l < plan.lcnt.size(); ++l) {
            hipLaunchKernelGGL(chol_diag_kernel<true>, dim3(plan.lcnt[l]), dim3(256), 0, st, A, n, 0,
                               plan.lcols + plan.lbeg[l], Winv, fail, x);
            if (plan.tcnt[l] > 0)
                hipLaunchKernelGGL(chol_level_update_kernel, dim3(4 * plan.tcnt[l]), dim3(256), 0, st, A, L, LT, n,
                                   Winv, plan.tasks + 4 * (int64_t)plan.tbeg[l], plan.contrib, fail, x);
        }
        return;
    }
    const int nblk = (n + NB - 1) / NB;
    for (int kb = 0; kb < nblk; ++kb) {
        const int k0 = kb * NB;
        hipLaunchKernelGGL(chol_diag_kernel<false>, dim3(1), dim3(256), 0, st, A, n, k0, nullptr, Winv, fail,
                           nullptr);
        const int m = plan.rcnt[kb];
        if (m > 0)
            hipLaunchKernelGGL(chol_panel_update_kernel, dim3(4 * (m * (m + 1) / 2)), dim3(256), 0, st, A, L, LT, n, k0, Winv,
                               plan.rows + plan.rbeg[kb], fail);
    }
}

// L y = rhs, then L^T x = y, both in one launch of one 1024-thread workgroup that walks the
// block columns forward and then backward: the factor couples each block to a few tiles, so a
// block step is a few thousand FMAs and a launch per step would cost more than the step.  The
// vector being solved for sits in LDS when it fits (kTrsvLds doubles), else in x itself; it holds
// the right-hand side, then y block by block, then the solution (x is zeroed instead if the
// factorisation failed).  The two sweeps are the same
// loop: block k takes u_k = M_k v_k in place of v_k, then v_i -= F_ik u_k for the tiles i listed
// for k, with M = W_kk, F = L (tile rows below k) forward and M = W_kk^T, F = L^T (tile columns
// left of k, read as rows of L^T) backward, so every product runs along rows: 16 lanes per row,
// 4 columns each, summed within the lanes' row by DPP.  The next step's M_k and first kTrsvPre
// tiles (listed per block, -1 padded, after the plan's counts) are fetched into registers while
// the current step runs: they do not depend on the vector, so only LDS traffic and barriers
// remain on the chain of steps.  A barrier also makes global writes before it visible to the
// whole workgroup.
constexpr int kTrsvLds = 16384;
constexpr int kTrsvPre = kCholPre;
constexpr int kTrsvLpr = 16;   // lanes per row of the products (per solve at n = 1800: 4 -> 393 us, 8 -> 240, 16 -> 192)

// Workgroup barrier that orders LDS accesses only: global loads issued before it stay in flight
// (__syncthreads() also waits for those).
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Lane permutations without LDS round trips.  DPP row_ror:n rotates each 16-lane row by n.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
constexpr int kRowRor8 = 0x128, kRowRor4 = 0x124;

constexpr int kHalfMirror = 0x141, kQuadXor2 = 0x4E, kQuadXor1 = 0xB1;

// Sum over each aligned group of G lanes (16: rotations of the 16-lane row by 8, 4, 2, 1; 8: the
// half-row mirror, which pairs lane i with 7 - i, then quad permutes xor 2 and xor 1; 4: the quad
// permutes), in every lane of the group.  Groups may be active or inactive as a whole.
template <int G>
__device__ __forceinline__ double group_sum(double u)
{
    if constexpr (G == 16) {
        u += dpp_f64<kRowRor8>(u);
        u += dpp_f64<kRowRor4>(u);
    } else if constexpr (G == 8) {
        u += dpp_f64<kHalfMirror>(u);
    }
    u += dpp_f64<kQuadXor2>(u);
    return u + dpp_f64<kQuadXor1>(u);
}

// Two doubles at p (16-byte aligned) if ok, else the two at `safe`, without a branch, so every
// call issues exactly one load and the compiler can count the loads still in flight (a select
// to zero would be placed right after the load and wait for it).  The callers skip a value that
// was not ok, or multiply it by an exact zero, and `safe` holds finite values.
__device__ __forceinline__ void load2_or_safe(const double *p, bool ok, double &a, double &b, const double *safe)
{
    const double2 v = *reinterpret_cast<const double2 *>(ok ? p : safe);
    a = v.x;
    b = v.y;
}

template <bool kInLds, int LPR>
__global__ void __launch_bounds__(64 * LPR) trsv_band_kernel(const double *__restrict__ L,
                                                         const double *__restrict__ LT,
                                                         const double *__restrict__ Winv, double *x, int n,
                                                         const int32_t *__restrict__ rows,
                                                         const int32_t *__restrict__ cols,
                                                         const int32_t *__restrict__ meta, const int32_t *fail)
{
    __shared__ double vs[kInLds ? kTrsvLds : 1];
    __shared__ double vk[NB];
    if (*fail) {   // no factor: the step is zero
        for (int e = threadIdx.x; e < n; e += blockDim.x) x[e] = 0.0;
        return;
    }
    double *v = kInLds ? vs : x;
    // with the vector in LDS the barriers need not wait for the prefetches
    auto sync = [] {
        if constexpr (kInLds) lds_barrier();
        else __syncthreads();
    };
    const int t = threadIdx.x, nblk = (n + NB - 1) / NB;
    const int32_t *rbeg = meta, *rcnt = meta + nblk, *cbeg = meta + 2 * nblk, *ccnt = meta + 3 * nblk;
    const int32_t *rpre = meta + 4 * nblk, *cpre = rpre + kTrsvPre * nblk;   // first tiles, -1 padded
    if (kInLds) {
        for (int e = t; e < n; e += blockDim.x) vs[e] = x[e];
        sync();
    }
    constexpr int CPL = NB / LPR;   // columns per lane
    const int row = t / LPR, c4 = (t % LPR) * CPL;   // thread = (row of the product, CPL columns)
    auto sweep = [&](const double *M, const double *F, const int32_t *pre, const int32_t *beg, const int32_t *cnt,
                     const int32_t *list, bool forward) {
        double wa[CPL], la[kTrsvPre][CPL], wb[CPL], lb[kTrsvPre][CPL];
        auto fetch = [&](int kb, double (&wn)[CPL], double (&ln)[kTrsvPre][CPL]) {
            const int k0 = kb * NB, nb = min(NB, n - k0);
            const double2 *Mr = reinterpret_cast<const double2 *>(M + ((int64_t)kb * NB + row) * NB + c4);
#pragma unroll
            for (int h = 0; h < CPL / 2; ++h) {   // the block is zero-padded
                const double2 m = Mr[h];
                wn[2 * h] = m.x;
                wn[2 * h + 1] = m.y;
            }
#pragma unroll
            for (int e = 0; e < kTrsvPre; ++e) {
                const int tile = pre[kTrsvPre * kb + e];
                const int i = tile >= 0 ? tile * NB + row : n;
#pragma unroll
                for (int h = 0; h < CPL / 2; ++h)   // columns c4 + 2 h, c4 + 2 h + 1 (nb is even)
                    load2_or_safe(F + (int64_t)i * n + k0 + c4 + 2 * h, i < n && c4 + 2 * h < nb, ln[e][2 * h],
                                  ln[e][2 * h + 1], M);
            }
        };
        auto step = [&](int kb, const double (&w)[CPL], const double (&l)[kTrsvPre][CPL]) {
            const int k0 = kb * NB, nb = min(NB, n - k0);
            double u = 0.0;
#pragma unroll
            for (int q = 0; q < CPL; ++q) u = fma(w[q], c4 + q < nb ? v[k0 + c4 + q] : 0.0, u);
            u = group_sum<LPR>(u);   // zero for rows beyond the block (M is zero-padded)
            const bool lead = t % LPR == 0;
            if (lead) vk[row] = u;
            sync();
            if (lead && row < nb) v[k0 + row] = u;
            double vq[CPL];
#pragma unroll
            for (int q = 0; q < CPL; ++q) vq[q] = vk[c4 + q];
#pragma unroll
            for (int e = 0; e < kTrsvPre; ++e) {
                const int tile = pre[kTrsvPre * kb + e];
                const int i = tile >= 0 ? tile * NB + row : n;
                if (i < n) {   // uniform over the row's lanes
                    double z = 0.0;
#pragma unroll
                    for (int q = 0; q < CPL; ++q) z = fma(l[e][q], vq[q], z);
                    z = group_sum<LPR>(z);
                    if (lead) v[i] -= z;
                }
            }
            for (int e = kTrsvPre; e < cnt[kb]; ++e) {
                const int i = list[beg[kb] + e] * NB + row;
                if (i >= n) continue;
                double z = 0.0;
#pragma unroll
                for (int q = 0; q < CPL; ++q)
                    if (c4 + q < nb) z = fma(F[(int64_t)i * n + k0 + c4 + q], vq[q], z);
                z = group_sum<LPR>(z);
                if (lead) v[i] -= z;
            }
            sync();
        };
        // Two steps per pass with the register sets swapped (static indexing keeps them in registers;
        // a copy out of the prefetch set would wait for its loads).  The fetches are unconditional
        // (past the end they repeat the last block), so that the loads in flight are the same on
        // every path and the waits for them can be counted.
        const int first = forward ? 0 : nblk - 1, dir = forward ? 1 : -1;
        auto clampb = [&](int kb) { return min(max(kb, 0), nblk - 1); };
        fetch(first, wa, la);
        for (int s = 0; s < nblk; s += 2) {
            const int kb = first + dir * s;
            fetch(clampb(kb + dir), wb, lb);
            step(kb, wa, la);
            if (s + 1 >= nblk) break;
            fetch(clampb(kb + 2 * dir), wa, la);
            step(kb + dir, wb, lb);
        }
    };
    sweep(Winv, L, rpre, rbeg, rcnt, rows, true);
    sweep(Winv + (int64_t)nblk * NB * NB, LT, cpre, cbeg, ccnt, cols, false);
    if (kInLds)
        for (int e = t; e < n; e += blockDim.x) x[e] = vs[e];
}

// One elimination-tree level of the triangular solves in a nested-dissection order, one workgroup
// per block column k of the level, gathering what the finished levels contribute (the library
// runs the forward sweep with the factorisation instead, and this kernel for the backward one):
//   forward   y_k = W_k (r_k - sum_j L_kj y_j)      over the tile columns j < k of block row k,
//   backward  x_k = W_k^T (y_k - sum_i L_ik^T x_i)  over the tile rows i > k of block column k,
// with F = L (tile (k, j)) or F = L^T (tile (k, i), rows of L^T) and M = W_k or W_k^T.  The tiles
// gathered belong to lower levels (forward) or higher ones (backward), finished by earlier
// launches.  Four lanes per row, 16 columns each; the sums of a row's lanes by quad permutes.
// x is zeroed instead if the factorisation failed.
__global__ void __launch_bounds__(256) trsv_level_kernel(const double *__restrict__ F, const double *__restrict__ M,
                                                         double *x, int n, const int32_t *__restrict__ lcols,
                                                         const int32_t *__restrict__ adj,
                                                         const int32_t *__restrict__ beg,
                                                         const int32_t *__restrict__ cnt, const int32_t *fail)
{
    __shared__ double sv[NB];
    const int kb = lcols[blockIdx.x], k0 = kb * NB;
    const int t = threadIdx.x, row = t >> 2, c16 = (t & 3) * 16;
    const bool lead = (t & 3) == 0;
    if (*fail) {
        if (t < NB) x[k0 + t] = 0.0;
        return;
    }
    double z = 0.0;
    const int b0 = beg[kb], m = cnt[kb];
    for (int e = 0; e < m; ++e) {
        const int j0 = adj[b0 + e] * NB;
        const double2 *Fr = reinterpret_cast<const double2 *>(F + (int64_t)(k0 + row) * n + j0 + c16);
        const double2 *xr = reinterpret_cast<const double2 *>(x + j0 + c16);
#pragma unroll
        for (int h = 0; h < 8; ++h) {
            const double2 f = Fr[h], v = xr[h];
            z = fma(f.x, v.x, z);
            z = fma(f.y, v.y, z);
        }
    }
    z = group_sum<4>(z);
    if (lead) sv[row] = x[k0 + row] - z;
    __syncthreads();
    const double2 *Mr = reinterpret_cast<const double2 *>(M + ((int64_t)kb * NB + row) * NB + c16);
    double u = 0.0;
#pragma unroll
    for (int h = 0; h < 8; ++h) {
        const double2 w = Mr[h];
        u = fma(w.x, sv[c16 + 2 * h], u);
        u = fma(w.y, sv[c16 + 2 * h + 1], u);
    }
    u = group_sum<4>(u);
    if (lead) x[k0 + row] = u;
}

void launch_chol_solve(const double *L, const double *LT, double *Winv, double *x, int n, const CholPlan &plan,
                       const int32_t *fail, hipStream_t st)
{
    if (plan.nd) {   // the forward substitution ran with the factorisation (launch_cholesky with x)
        const int nblk = n / NB, nlev = (int)plan.lcnt.size();
        const int32_t *rbeg = plan.meta, *rcnt = rbeg + nblk;
        for (int l = nlev - 1; l >= 0; --l)
            hipLaunchKernelGGL(trsv_level_kernel, dim3(plan.lcnt[l]), dim3(256), 0, st, LT,
                               Winv + (int64_t)nblk * NB * NB, x, n, plan.lcols + plan.lbeg[l], plan.rows, rbeg,
                               rcnt, fail);
        return;
    }
    // PBA_TRSV_LDS_MAX (doubles, at most kTrsvLds) lowers the size up to which the vector is kept
    // in LDS; 0 selects the global-memory variant for every size.  PBA_TRSV_LPR (4, 8 or 16) sets
    // the lanes per row of the products.
    int lds_max = kTrsvLds, lpr = kTrsvLpr;
    if (const char *e = std::getenv("PBA_TRSV_LDS_MAX")) lds_max = std::min(kTrsvLds, std::max(0, std::atoi(e)));
    if (const char *e = std::getenv("PBA_TRSV_LPR")) lpr = std::atoi(e);
    const bool in_lds = n <= lds_max;
#define PBA_TRSV_LAUNCH(LDS, G)                                                                                 \
    hipLaunchKernelGGL((trsv_band_kernel<LDS, G>), dim3(1), dim3(64 * G), 0, st, L, LT, Winv, x, n, plan.rows, \
                       plan.cols, plan.meta, fail)
    if (lpr == 4) {
        if (in_lds) PBA_TRSV_LAUNCH(true, 4);
        else PBA_TRSV_LAUNCH(false, 4);
    } else if (lpr == 16) {
        if (in_lds) PBA_TRSV_LAUNCH(true, 16);
        else PBA_TRSV_LAUNCH(false, 16);
    } else {
        if (in_lds) PBA_TRSV_LAUNCH(true, 8);
        else PBA_TRSV_LAUNCH(false, 8);
    }
#undef PBA_TRSV_LAUNCH
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
// off: first element of each pose's 6 in dx (a nested-dissection solve's layout), nullptr = 6 k.
__global__ void __launch_bounds__(256) boxplus_kernel(const double *__restrict__ X, const double *__restrict__ dx,
                                                      const int32_t *__restrict__ off, double *__restrict__ Xo,
                                                      int N, const int32_t *fail, LmState *lm)
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
        const double *d = dx + (off ? (int64_t)off[k] : 6 * (int64_t)k);
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

void launch_boxplus(const double *X, const double *dx, const int32_t *off, double *Xout, int N, const int32_t *fail,
                    LmState *lm, hipStream_t st)
{
    hipLaunchKernelGGL(boxplus_kernel, dim3(1), dim3(256), 0, st, X, dx, off, Xout, N, fail, lm);
}

// dst[6 k + i] = src[off[k] + i]: a nested-dissection solve's step in pose order.
__global__ void gather_step_kernel(double *__restrict__ dst, const double *__restrict__ src,
                                   const int32_t *__restrict__ off, int N)
{
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < 6 * N; e += gridDim.x * blockDim.x)
        dst[e] = src[off[e / 6] + e % 6];
}

void launch_gather_step(double *dst, const double *src, const int32_t *off, int N, hipStream_t st)
{
    const int blocks = std::max(1, std::min(1024, (6 * N + 255) / 256));
    hipLaunchKernelGGL(gather_step_kernel, dim3(blocks), dim3(256), 0, st, dst, src, off, N);
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
    double *log_row = logbuf + kLogRow * (int64_t)min(lm->iter, log_cap - 1);
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
    // the last launch of an iteration: its end stamp
    reinterpret_cast<uint64_t *>(log_row)[9] = (uint64_t)wall_clock64();
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
// log row: the evaluation inside a captured iteration is bracketed by two of these (which = 0, 1)
// and the iteration starts with one (which = 2), so every replay of the graph leaves its own
// durations.
__global__ void stamp_kernel(const LmState *lm, double *logbuf, int log_cap, int which)
{
    if (threadIdx.x != 0) return;
    uint64_t *row = reinterpret_cast<uint64_t *>(logbuf + kLogRow * (int64_t)min(lm->iter, log_cap - 1));
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
