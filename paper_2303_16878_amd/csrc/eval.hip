// Evaluation kernels: pair setup, per-pixel residuals/Jacobians/accumulation over a
// persistent work queue, ordered per-pair reduction, pair expansion and assembly of
// the 6N x 6N normal equations.
//
// Paper: warp Eq. (uprime) and objective Eq. (total-error-multicue) in Sec. IV-C;
// projections in Sec. III; Jacobians, cue maps and sensor offsets in the
// supplementary material.
//
// Frames.  For pair (s, t) the kernel works in the target *sensor* frame:
//   q      = pi_s^-1(u, d)                   source sensor frame
//   p_bar  = R q + t                          target sensor frame, with
//   R      = R_ot^T R_t^T R_s R_os,  t = R_ot^T (R_t^T (R_s t_os + t_s - t_t) - t_ot)
// and differentiates with respect to the target-pose perturbation expressed in the
// target sensor axes, dx' = D dx_t with D = blockdiag(R_ot^T, R_ot^T):
//   d p_bar / d dx' = [-I | 2 [y'']_x],  y'' = p_bar + R_ot^T t_ot
// (the supplementary's -R_o^T [I  2 skewp(y)] rotated into sensor axes; skewp(v) w = w x v).
// Rows for the platform perturbations follow per pair in FP64:
//   J_t = J' D,   J_s = J_t A = J' (D A),  A = [[-R, 2 skewp(t) R], [0, -R]]
// with (R, t) = X_t^-1 X_s; A is the exact algebraic relation between the two
// supplementary point Jacobians.  So per pixel only the 6-vector J' of each cue
// row is formed and 21 + 6 unique products are accumulated.

#include "pba_internal.h"

#include <type_traits>

namespace pba {

// ------------------------------------------------------------------ pair setup (FP64)

__device__ static inline void mm3(const double *A, const double *B, double *C) {
    double T[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) T[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
    for (int i = 0; i < 9; ++i) C[i] = T[i];
}
__device__ static inline void mtm3(const double *A, const double *B, double *C) {   // A^T B
    double T[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) T[3 * i + j] = A[i] * B[j] + A[3 + i] * B[3 + j] + A[6 + i] * B[6 + j];
    for (int i = 0; i < 9; ++i) C[i] = T[i];
}
__device__ static inline void mv3(const double *A, const double *v, double *o) {
    double r0 = A[0] * v[0] + A[1] * v[1] + A[2] * v[2];
    double r1 = A[3] * v[0] + A[4] * v[1] + A[5] * v[2];
    double r2 = A[6] * v[0] + A[7] * v[1] + A[8] * v[2];
    o[0] = r0; o[1] = r1; o[2] = r2;
}
__device__ static inline void mtv3(const double *A, const double *v, double *o) {   // A^T v
    double r0 = A[0] * v[0] + A[3] * v[1] + A[6] * v[2];
    double r1 = A[1] * v[0] + A[4] * v[1] + A[7] * v[2];
    double r2 = A[2] * v[0] + A[5] * v[1] + A[8] * v[2];
    o[0] = r0; o[1] = r1; o[2] = r2;
}

__global__ void pair_setup_kernel(const double *__restrict__ poses, const int2 *__restrict__ pairs, int P,
                                  const SensorDev *__restrict__ sensors, const KfDev *__restrict__ kfs,
                                  PairDev *__restrict__ out, uint32_t *counters, int ncounters)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < ncounters) counters[(int64_t)p * kCtrStride] = 0u;
    if (p >= P) return;
    const int s = pairs[p].x, t = pairs[p].y;
    const SensorDev &ss = sensors[kfs[s].sensor];
    const SensorDev &st = sensors[kfs[t].sensor];
    const double *Rs = poses + 12 * (int64_t)kfs[s].pose, *ts = Rs + 9;
    const double *Rt = poses + 12 * (int64_t)kfs[t].pose, *tt = Rt + 9;
    // platform-level relative pose X_t^-1 X_s
    double Rp[9], tp[3], d3[3];
    mtm3(Rt, Rs, Rp);
    for (int k = 0; k < 3; ++k) d3[k] = ts[k] - tt[k];
    mtv3(Rt, d3, tp);
    // sensor-to-sensor transform
    double M[9], R[9], tv[3], tw[3];
    mm3(Rp, ss.Ro, M);
    mtm3(st.Ro, M, R);
    mv3(Rp, ss.to, tw);
    for (int k = 0; k < 3; ++k) tw[k] += tp[k] - st.to[k];
    mtv3(st.Ro, tw, tv);
    double c[3];
    mtv3(st.Ro, st.to, c);
    PairDev &o = out[p];
    for (int k = 0; k < 9; ++k) o.Rd[k] = R[k];
    for (int k = 0; k < 3; ++k) {
        o.td[k] = tv[k];
        o.c[k] = (float)c[k];
    }
    // D = R_ot^T ; A = [[-Rp, 2 skewp(tp) Rp], [0, -Rp]] ; E = blockdiag(D, D) A
    double D[9];
    for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) D[3 * i + j] = st.Ro[3 * j + i];
    for (int k = 0; k < 9; ++k) o.D[k] = D[k];
    const double Sp[9] = {0, tp[2], -tp[1], -tp[2], 0, tp[0], tp[1], -tp[0], 0};
    double A12[9], DR[9], DA12[9];
    mm3(Sp, Rp, A12);
    for (int k = 0; k < 9; ++k) A12[k] *= 2.0;
    mm3(D, Rp, DR);
    mm3(D, A12, DA12);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            o.E[6 * i + j] = -DR[3 * i + j];
            o.E[6 * i + 3 + j] = DA12[3 * i + j];
            o.E[6 * (3 + i) + j] = 0.0;
            o.E[6 * (3 + i) + 3 + j] = -DR[3 * i + j];
        }
    o.src = s;
    o.tgt = t;
}

void launch_pair_setup(const double *poses, const int2 *pairs, int P, const SensorDev *sensors, const KfDev *kfs,
                       PairDev *out, uint32_t *counters, int ncounters, hipStream_t st)
{
    const int n = P > ncounters ? P : ncounters;
    hipLaunchKernelGGL(pair_setup_kernel, dim3((n + 127) / 128), dim3(128), 0, st, poses, pairs, P, sensors, kfs,
                       out, counters, ncounters);
}

// ------------------------------------------------------------------ per-pixel evaluation

// 1/x and 1/sqrt(x) for x > 0 (finite): in FP32 the hardware reciprocal and reciprocal square root
// (about 1 ulp), where they feed Jacobians and weights whose own FP32 rounding is of the same
// order; in FP64 the hardware estimates (relative error below 2^-24) refined by two Newton steps,
// within a few ulps (an IEEE division or square root costs several times the instructions).
template <typename T>
__device__ __forceinline__ T fast_rcp(T x);
template <>
__device__ __forceinline__ float fast_rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <>
__device__ __forceinline__ double fast_rcp<double>(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}
template <typename T>
__device__ __forceinline__ T fast_rsq(T x);
template <>
__device__ __forceinline__ float fast_rsq<float>(float x) { return __builtin_amdgcn_rsqf(x); }
template <>
__device__ __forceinline__ double fast_rsq<double>(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    y = y * fma(-0.5 * x * y, y, 1.5);
    return y * fma(-0.5 * x * y, y, 1.5);
}

// 1/x in FP64: the hardware estimate (relative error below 2^-24, measured on this target) refined
// by one Newton step, which squares the error: below 3e-15.  The geometry needs far less (a
// projected coordinate of 2000 px then carries ~1e-11 px).
__device__ __forceinline__ double rcp_f64(double x)
{
    const double r = __builtin_amdgcn_rcp(x);
    return fma(r, fma(-x, r, 1.0), r);
}

// sqrt(x) for x > 0 in FP64: x times the hardware reciprocal square root (below 2^-24) refined by
// one Newton step: relative error below 5e-15 (3e-13 m at 80 m range).
__device__ __forceinline__ double sqrt_f64(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    y = y * fma(-0.5 * x * y, y, 1.5);
    return x * y;
}

// Coarse atan2 in FP32 (error below 6.1e-4 rad): octant reduction and a quadratic in t^2 fitted
// to atan on [0, 1].  It only picks the nearest ray of a table, so a fraction of a pixel is enough.
__device__ __forceinline__ float atan2_coarse(float y, float x)
{
    const float ax = fabsf(x), ay = fabsf(y);
    const float mx = fmaxf(fmaxf(ax, ay), 1e-30f), mn = fminf(ax, ay);
    const float t = mn * __builtin_amdgcn_rcpf(mx), s = t * t;
    float a = t * fmaf(fmaf(0.07933887839317322f, s, -0.28869009017944336f), s, 0.9953579306602478f);
    if (ay > ax) a = 1.57079637f - a;
    if (x < 0.f) a = 3.14159274f - a;
    return y < 0.f ? -a : a;
}

// atan(t) for |t| <= 1 by the same quadratic in t^2 (error below 6.1e-4 rad)
__device__ __forceinline__ float atan_unit(float t)
{
    const float s = t * t;
    return t * fmaf(fmaf(0.07933887839317322f, s, -0.28869009017944336f), s, 0.9953579306602478f);
}

// atan(t) for small |t| by its Taylor series to t^5 (remainder below t^7 / 7: 2.4e-19 rad at 3e-3,
// about the largest offset from the nearest ray of a 2048 x 128 spherical image; 1.1e-10 rad at
// 0.05, the offset of a 64-column image).
__device__ __forceinline__ double atan_small(double t)
{
    const double t2 = t * t;
    return t * fma(t2, fma(t2, 0.2, -1.0 / 3.0), 1.0);
}


// value and image Jacobian [d/dcol, d/drow] of one channel at the bilinear point.
// a0..a3: row y0, cols x0-1..x0+2; b0..b3: row y0+1; c1,c2: row y0-1, cols x0, x0+1;
// d1,d2: row y0+2, cols x0, x0+1.
template <typename T, int GM>
__device__ __forceinline__ void sample_grad(T a0, T a1, T a2, T a3, T b0, T b1, T b2, T b3, T c1, T c2, T d1, T d2,
                                            T w00, T w01, T w10, T w11, T al, T be, T &Gx, T &Gy)
{
    if (GM == 0) {
        // central differences 1/2 (I[x+1] - I[x-1]) at each tap, blended with the bilinear weights;
        // returned without the factor 1/2, which the caller folds into the projective Jacobian
        // (scaling by 1/2 is exact, so the products are the same)
        Gx = w00 * (a2 - a0) + w01 * (a3 - a1) + w10 * (b2 - b0) + w11 * (b3 - b1);
        Gy = w00 * (b1 - c1) + w01 * (b2 - c2) + w10 * (d1 - a1) + w11 * (d2 - a2);
    } else {
        Gx = (T(1) - be) * (a2 - a1) + be * (b2 - b1);
        Gy = (T(1) - al) * (b1 - a1) + al * (b2 - a2);
    }
}
template <typename T, int GM>
__device__ __forceinline__ void sample_channel(T a0, T a1, T a2, T a3, T b0, T b1, T b2, T b3, T c1, T c2, T d1,
                                               T d2, T w00, T w01, T w10, T w11, T al, T be, T &V, T &Gx, T &Gy)
{
    V = w00 * a1 + w01 * a2 + w10 * b1 + w11 * b2;
    sample_grad<T, GM>(a0, a1, a2, a3, b0, b1, b2, b3, c1, c2, d1, d2, w00, w01, w10, w11, al, be, Gx, Gy);
}

// Per-pixel sums of one cue row into v: v[0..20] += om J_i J_j (upper triangle, row-major),
// v[21..26] += om e J_i.  The five rows of a pixel are summed in the evaluation precision; the sums
// of the 64 pixels of a wave are then added by a fixed butterfly (wave_reduce_scatter) and the wave
// totals accumulated in FP64.  Summation depth is log2 of the terms, not their number: the
// source-pose blocks are expanded from these sums by A, whose lever arm (the pair baseline)
// amplifies relative errors by up to ~|t|^2 / range^2, and sequential FP32 sums over many pixels
// would not hold the 1e-5 agreement on long baselines.
// FP64 path: the same 27 sums per lane straight into FP64 accumulators (each product exact, each
// addition rounded once), no butterfly.
__device__ __forceinline__ void accumulate_row(double *acc, const double (&J)[6], double e, double om)
{
    double wj[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) wj[i] = om * J[i];
    int idx = 0;
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = i; j < 6; ++j) { acc[idx] = fma(wj[i], J[j], acc[idx]); ++idx; }
#pragma unroll
    for (int i = 0; i < 6; ++i) acc[ACC_B + i] = fma(wj[i], e, acc[ACC_B + i]);
}

template <typename T>
__device__ __forceinline__ void add_row(T (&v)[32], const T (&J)[6], T e, T om)
{
    T wj[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) wj[i] = om * J[i];
    int idx = 0;
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = i; j < 6; ++j) { v[idx] = fma(wj[i], J[j], v[idx]); ++idx; }
#pragma unroll
    for (int i = 0; i < 6; ++i) v[ACC_B + i] = fma(wj[i], e, v[ACC_B + i]);
}

template <typename T>
__device__ __forceinline__ void add_cue_row(T (&v)[32], double *acc64, const T (&J)[6], T e, T om)
{
    if constexpr (std::is_same<T, float>::value) add_row(v, J, e, om);
    else accumulate_row(acc64, J, e, om);
}

// Exchange lanes 32..63 of x with lanes 0..31 of y, and the odd 16-lane rows of x with the even
// rows of y (whole-register lane permutations, no memory).
__device__ __forceinline__ void swap_half(float &x, float &y)
{
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false, false);
    x = __uint_as_float(r[0]);
    y = __uint_as_float(r[1]);
}
__device__ __forceinline__ void swap_row(float &x, float &y)
{
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y), false, false);
    x = __uint_as_float(r[0]);
    y = __uint_as_float(r[1]);
}
__device__ __forceinline__ void swap_half(double &x, double &y)
{
    float xl = __int_as_float(__double2loint(x)), xh = __int_as_float(__double2hiint(x));
    float yl = __int_as_float(__double2loint(y)), yh = __int_as_float(__double2hiint(y));
    swap_half(xl, yl);
    swap_half(xh, yh);
    x = __hiloint2double(__float_as_int(xh), __float_as_int(xl));
    y = __hiloint2double(__float_as_int(yh), __float_as_int(yl));
}
__device__ __forceinline__ void swap_row(double &x, double &y)
{
    float xl = __int_as_float(__double2loint(x)), xh = __int_as_float(__double2hiint(x));
    float yl = __int_as_float(__double2loint(y)), yh = __int_as_float(__double2hiint(y));
    swap_row(xl, yl);
    swap_row(xh, yh);
    x = __hiloint2double(__float_as_int(xh), __float_as_int(xl));
    y = __hiloint2double(__float_as_int(yh), __float_as_int(yl));
}

// Sum 32 per-lane values over the 64 lanes of a wave.  Butterfly reduce-scatter: at each step a
// lane keeps one half of its values and adds its partner's copy of that half (partners l ^ 32,
// l ^ 16, l ^ 8, l ^ 7, l ^ 2; each partner differs from the lane in the bit that chooses the
// half, and the five masks span all 64 lanes); finally lanes 2k and 2k + 1 add their totals.
// Returns the wave total of value k = lane >> 1 (the same in both lanes of the pair).
template <typename T>
__device__ __forceinline__ T wave_reduce_scatter(T (&v)[32], int lane)
{
#pragma unroll
    for (int i = 0; i < 16; ++i) { T x = v[i], y = v[i + 16]; swap_half(x, y); v[i] = x + y; }
#pragma unroll
    for (int i = 0; i < 8; ++i) { T x = v[i], y = v[i + 8]; swap_row(x, y); v[i] = x + y; }
#pragma unroll
    for (int m = 8, n = 4; n >= 1; m >>= 1, n >>= 1) {
        const bool up = (lane & m) != 0;
        const int pm = m == 4 ? 7 : m;
#pragma unroll
        for (int i = 0; i < n; ++i) {
            const T keep = up ? v[i + n] : v[i], send = up ? v[i] : v[i + n];
            v[i] = keep + __shfl_xor(send, pm, 64);
        }
    }
    return v[0] + __shfl_xor(v[0], 1, 64);
}

// Lane permutations inside 16-lane rows (DPP): xor 8 = rotate the row by 8, xor 7 = mirror each
// half-row, xor 2 and xor 1 = quad permutations [2,3,0,1] and [1,0,3,2].
constexpr int kDppXor8 = 0x128, kDppXor7 = 0x141, kDppXor2 = 0x4E, kDppXor1 = 0xB1;
template <int CTRL>
__device__ __forceinline__ float dpp(float x)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xF, 0xF, true));
}
// (m & a) | (~m & b) for an all-ones / all-zeros lane mask m (one bit-field insert)
__device__ __forceinline__ float bsel(uint32_t m, float a, float b)
{
    return __uint_as_float((m & __float_as_uint(a)) | (~m & __float_as_uint(b)));
}
// Lane mask of bit `b` of the lane index, opaque to the compiler: a visible boolean would be
// turned back into per-value selects (and, over several steps, into chains of compares).
template <int B>
__device__ __forceinline__ uint32_t lane_bit_mask(int lane)
{
    uint32_t r;
    asm volatile("v_bfe_i32 %0, %1, %2, 1" : "=v"(r) : "v"(lane), "i"(B));
    return r;
}

template <>
__device__ __forceinline__ float wave_reduce_scatter<float>(float (&v)[32], int lane)
{
#pragma unroll
    for (int i = 0; i < 16; ++i) { float x = v[i], y = v[i + 16]; swap_half(x, y); v[i] = x + y; }
#pragma unroll
    for (int i = 0; i < 8; ++i) { float x = v[i], y = v[i + 8]; swap_row(x, y); v[i] = x + y; }
    const uint32_t m3 = lane_bit_mask<3>(lane), m2 = lane_bit_mask<2>(lane), m1 = lane_bit_mask<1>(lane);
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = bsel(m3, v[i + 4], v[i]) + dpp<kDppXor8>(bsel(m3, v[i], v[i + 4]));
#pragma unroll
    for (int i = 0; i < 2; ++i) v[i] = bsel(m2, v[i + 2], v[i]) + dpp<kDppXor7>(bsel(m2, v[i], v[i + 2]));
    v[0] = bsel(m1, v[1], v[0]) + dpp<kDppXor2>(bsel(m1, v[0], v[1]));
    return v[0] + dpp<kDppXor1>(v[0]);
}

// J' of a cue row whose point-space derivative is a = d e / d p_bar (up to sign conventions below):
// J' = [-a ; 2 a x y'']  (translation, rotation), plus an optional rotation-only term z.
template <typename T>
__device__ __forceinline__ void row_from_a(T (&J)[6], T ax, T ay, T az, T y2x, T y2y, T y2z)
{
    J[0] = -ax;
    J[1] = -ay;
    J[2] = -az;
    J[3] = ay * y2z - az * y2y;
    J[4] = az * y2x - ax * y2z;
    J[5] = ax * y2y - ay * y2x;
}

template <typename T>
struct Lut;
template <>
struct Lut<float> {
    typedef float2 type;
    __device__ static const float2 *ptr(const EvalArgs &a) { return a.lut32; }
};
template <>
struct Lut<double> {
    typedef double2 type;
    __device__ static const double2 *ptr(const EvalArgs &a) { return a.lut64; }
};

// Per-wave queue of valid correspondences found by phase 1b, consumed by phase 2.
// Structure of arrays, 128 slots per wave (a chunk appends at most 64; phase 2 drains 64 at a time).
constexpr int kQ = 128;
template <typename T>
struct WaveQueue {
    int pix[kQ];
    int cell[kQ];          // x0 | y0 << 16
    T al[kQ], be[kQ];      // bilinear fractions
    T px[kQ], py[kQ], pz[kQ];   // p_bar
    T ed[kQ], gxd[kQ], gyd[kQ]; // depth residual and depth-channel image Jacobian
};

// Per-wave queue of the points that pass phase 1a (the first projection and the depth-interval test),
// consumed 64 at a time by phase 1b: the pixel, the first projection's table column and row, and the point
// in the target sensor frame (FP64).
struct WaveQueueA {
    int pix[kQ];
    int kcr[kQ];           // column | row << 16; debug launches: bit 15 = interval test passed, bit 31 = near
    double X[kQ], Y[kQ], Z[kQ];
};

// b-only accumulation for the loss adjoint, per lane in FP64: acc[i] += om * e * J_i
template <typename T>
__device__ __forceinline__ void accumulate_row_b(double *acc, const T (&J)[6], T e, T om)
{
    const double ome = (double)om * (double)e;
#pragma unroll
    for (int i = 0; i < 6; ++i) acc[i] = fma(ome, (double)J[i], acc[i]);
}

// Bounds-checked loads from one keyframe plane through a buffer resource: 32-bit byte offsets,
// the stencil's row steps in a scalar offset and its column steps in the instruction's immediate
// offset, so the 12 taps cost one address computation.  kRawBufferWord3 is the descriptor's
// fourth word for raw 32-bit element access on this target family (out-of-range loads return 0).
constexpr int kRawBufferWord3 = 0x00020000;
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
// Per-pair constants (pose product, sensor intrinsics, thresholds) are the same in every lane:
// readfirstlane pins them to scalar registers, which frees about 30 vector registers and lets the
// spherical FP32 kernel run four waves per SIMD instead of three.
__device__ __forceinline__ float uni_f(float v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))); }
__device__ __forceinline__ double uni_d(double v)
{
    return __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(v)), __builtin_amdgcn_readfirstlane(__double2loint(v)));
}
// A register whose contents do not matter (an empty asm statement defines it): for values that
// are only read on paths that set them, without instructions that clear them on the others.
template <typename V>
__device__ __forceinline__ V any_value()
{
    V x;
    asm volatile("" : "=v"(x));
    return x;
}
template <typename P>
__device__ __forceinline__ const P *uni_ptr(const P *p)
{
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return (const P *)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void *p, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, kRawBufferWord3);
}
__device__ __forceinline__ float ld_f32(__amdgpu_buffer_rsrc_t r, int voff, int soff)
{
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
// BF16 texels: {I, nx, ny, nz} in two dwords (low half first), or one 16-bit intensity
__device__ __forceinline__ float4 ld_bf16x4(__amdgpu_buffer_rsrc_t r, int voff, int soff)
{
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
    return make_float4(__uint_as_float(v[0] << 16), __uint_as_float(v[0] & 0xFFFF0000u), __uint_as_float(v[1] << 16),
                       __uint_as_float(v[1] & 0xFFFF0000u));
}
__device__ __forceinline__ float ld_bf16(__amdgpu_buffer_rsrc_t r, int voff, int soff)
{
    return bf16_to_f32((uint32_t)__builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0));
}
__device__ __forceinline__ float2 ld_f32x2(__amdgpu_buffer_rsrc_t r, int voff)
{
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, 0, 0);
    return make_float2(__uint_as_float(v[0]), __uint_as_float(v[1]));
}
__device__ __forceinline__ double2 ld_f64x2(__amdgpu_buffer_rsrc_t r, int voff)
{
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, voff, 0, 0);
    return make_double2(__hiloint2double((int)v[1], (int)v[0]), __hiloint2double((int)v[3], (int)v[2]));
}
__device__ __forceinline__ float4 ld_f32x4(__amdgpu_buffer_rsrc_t r, int voff, int soff)
{
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
    return make_float4(__uint_as_float(v[0]), __uint_as_float(v[1]), __uint_as_float(v[2]), __uint_as_float(v[3]));
}

// The 12-tap stencil around cell (x0, y0), in the order the sampling expects: row y0 cols
// x0-1..x0+2, row y0+1 cols x0-1..x0+2, row y0-1 cols x0, x0+1, row y0+2 cols x0, x0+1.
// `voff` addresses (x0 - 1, y0 - 1); `rowb` is one image row in bytes; E the element size.
template <typename V, int E, typename L>
__device__ __forceinline__ void load_stencil(V (&t)[12], L ld, int voff, int rowb)
{
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        t[c] = ld(voff + c * E, rowb);
        t[4 + c] = ld(voff + c * E, 2 * rowb);
    }
    t[8] = ld(voff + E, 0);
    t[9] = ld(voff + 2 * E, 0);
    t[10] = ld(voff + E, 3 * rowb);
    t[11] = ld(voff + 2 * E, 3 * rowb);
}

// ADJ: the loss adjoint -- only b (gradient) is accumulated, and dF/d(image) is scattered into
// the gradient arenas with hardware float atomics.
// ZB: the z-buffer occlusion variant (a separate instantiation, so the plain evaluation carries
// none of its code).
// BF: intensity and normal planes stored as BF16 (a separate instantiation; FP32 path only).
template <typename T, int NCH, int SM, int TM, int GM, bool DBG, bool ADJ = false, bool ZB = false, bool BF = false>
__global__ void __launch_bounds__(kBlock)
    // two cues between pinhole sensors (FP32): six waves per SIMD (80 VGPRs), which the register allocator
    // would otherwise miss by one
    __attribute__((amdgpu_waves_per_eu(
        std::is_same<T, float>::value && !DBG && !ADJ && NCH == 2 && SM == MODEL_PINHOLE && TM == MODEL_PINHOLE ? 6
                                                                                                             : 1)))
    eval_kernel(EvalArgs a, int item_base, int n_items)
{
    __shared__ WaveQueue<T> s_q[kBlock / 64];
    __shared__ WaveQueueA s_qa[kBlock / 64];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave index: uniform
    WaveQueue<T> &Q = s_q[wave];
    WaveQueueA &QA = s_qa[wave];
    typedef typename Lut<T>::type L2;
    const L2 *lut = Lut<T>::ptr(a);
    constexpr bool F32 = std::is_same<T, float>::value;

    // The items of a launch form kXcd contiguous queues; workgroups are dispatched round-robin
    // over the XCDs, so the waves of workgroup w drain queue w % kXcd first (items that share target
    // images stay on one XCD's L2), then help with the others.  Each wave takes items on its own
    // and leaves once all queues are exhausted: no wave waits for another.
    int q = 0;   // lane 0: queues tried so far
    for (;;) {
        int got = -1;
        if (lane == 0) {
            while (q < kXcd) {
                const int x = ((int)blockIdx.x + q) % kXcd;
                const int lo = (int)((int64_t)n_items * x / kXcd), hi = (int)((int64_t)n_items * (x + 1) / kXcd);
                // a plain read first: an exhausted queue costs no atomic (thousands of waves leave at the end)
                uint32_t *const ctr = a.counter + x * kCtrStride;
                const uint32_t seen = __hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (seen < (uint32_t)(hi - lo)) {
                    const int v = (int)atomicAdd(ctr, 1u);
                    if (v < hi - lo) { got = lo + v; break; }
                }
                ++q;
            }
        }
        const int it = __builtin_amdgcn_readfirstlane(got);   // lane 0's
        if (it < 0) break;
        const int item = a.item_map ? a.item_map[item_base + it] : item_base + it;
        const int pair = __builtin_amdgcn_readfirstlane(a.item_pair[item]);
        const int px0 = __builtin_amdgcn_readfirstlane(a.item_px0[item]);
        const PairDev &pd = a.pairs[pair];
        const KfDev ks = a.kfs[pd.src], kt = a.kfs[pd.tgt];
        const SensorDev &ss = a.sensors[ks.sensor];
        const SensorDev &st = a.sensors[kt.sensor];
        // per-item values are the same in every lane: keep them in scalar registers (buffer
        // resources and scalar offsets must be)
        const int Ws = uni(ss.W), npx = uni(ss.npx), Wt = uni(st.W), Ht = uni(st.H);
        const uint32_t magic = (uint32_t)uni((int)ss.magic_w);
        const int px1 = min(px0 + a.items_px, npx);

        // pair transform in FP64 (phase 1 geometry, the normal cue's rotation, adjoint terms)
        double Rd[9], td[3];
#pragma unroll
        for (int k = 0; k < 9; ++k) Rd[k] = uni_d(pd.Rd[k]);
#pragma unroll
        for (int k = 0; k < 3; ++k) td[k] = uni_d(pd.td[k]);
        T cc[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) cc[k] = (T)uni_f(pd.c[k]);
        if (!F32) {
            double cd[3];
            mtv3(st.Ro, st.to, cd);
            for (int k = 0; k < 3; ++k) cc[k] = (T)cd[k];
        }
        const double st_fx = uni_d(st.fxd), st_fy = uni_d(st.fyd), st_cx = uni_d(st.cxd), st_cy = uni_d(st.cyd), st_dmin = uni_d(st.dmind);
        // focal lengths of the projective Jacobian, halved for central differences (see sample_grad)
        const T fx = (T)(GM == 0 ? 0.5 * st_fx : st_fx), fy = (T)(GM == 0 ? 0.5 * st_fy : st_fy);
        const double taud_gate = uni_d(st.taud);   // occlusion bound, FP64 in both paths
        const T om_g = (T)a.omega_g, om_d = (T)a.omega_d, om_n = (T)a.omega_n, delta = (T)a.huber;
        // ray-table offsets of the source (unprojection) and target (projection) sensors in scalar
        // registers: read once per item, not from the sensor record in every chunk
        const int s_lcol = uni(ss.lut_col), s_lrow = uni(ss.lut_row);
        const int t_lcol = uni(st.lut_col), t_lrow = uni(st.lut_row);
        const L2 *lcol = lut + s_lcol, *lrow = lut + s_lrow;
        // z-buffer occlusion variant: this pair's source z-buffer (FP32 depth bits per target cell)
        uint32_t *const zb = ZB ? a.zbuf + a.zoff[pair] : nullptr;
        const uint32_t tnpx = (uint32_t)Ht * (uint32_t)Wt;
        const __amdgpu_buffer_rsrc_t r_tdep = plane_rsrc(uni_ptr(a.dep + kt.off), tnpx * 4u);
        const __amdgpu_buffer_rsrc_t r_sdep = plane_rsrc(uni_ptr(a.dep + ks.off), (uint32_t)npx * 4u);
        // the source keyframe's attribute plane (its own texels of the queued pixels)
        const uint32_t att_e = NCH == 5 ? (BF ? 8u : 16u) : (BF ? 2u : 4u);
        const __amdgpu_buffer_rsrc_t r_satt =
            NCH == 5 ? (BF ? plane_rsrc(uni_ptr(a.att4h + ks.off), (uint32_t)npx * att_e)
                           : plane_rsrc(uni_ptr(a.att4 + ks.off), (uint32_t)npx * att_e))
                     : (BF ? plane_rsrc(uni_ptr(a.att1h + ks.off), (uint32_t)npx * att_e)
                           : plane_rsrc(uni_ptr(a.att1 + ks.off), (uint32_t)npx * att_e));
        const __amdgpu_buffer_rsrc_t r_lut = plane_rsrc(uni_ptr(a.lut64), (uint32_t)a.lut64_bytes);
        const __amdgpu_buffer_rsrc_t r_gate = plane_rsrc(uni_ptr(a.gate + kt.off), tnpx * 8u);
        // uniform flags as one scalar word.  Bit 0: the depth-interval test runs (spherical targets whose first
        // projection is within half a pixel, and not in the z-buffer fill pass, which needs every point inside
        // the image).  Bit 1: the division-free coarse elevation.
        const int flags = uni((TM == MODEL_SPHERICAL && st.early != 0 && !(ZB && a.zpass) ? 1 : 0) | (st.el45 != 0 ? 2 : 0));
        const __amdgpu_buffer_rsrc_t r_tatt =
            NCH == 5 ? (BF ? plane_rsrc(uni_ptr(a.att4h + kt.off), tnpx * 8u) : plane_rsrc(uni_ptr(a.att4 + kt.off), tnpx * 16u))
                     : (BF ? plane_rsrc(uni_ptr(a.att1h + kt.off), tnpx * 2u) : plane_rsrc(uni_ptr(a.att1 + kt.off), tnpx * 4u));

        // FP64 accumulators: lanes 2k, 2k + 1 hold this wave's total of H/b sum k (k < 27); rho per
        // lane; the adjoint keeps b per lane
        double acc_hb = 0.0, acc_F = 0.0, acc_b[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        double acc64[F32 ? 1 : ACC_F];   // FP64 path: the 27 sums per lane
#pragma unroll
        for (int k = 0; k < (F32 ? 1 : ACC_F); ++k) acc64[k] = 0.0;
        int n_valid = 0;               // per lane
        int n_eval = 0;                // per wave
        int n_band = 0;                // per wave
        int headA = 0, tailA = 0, head = 0, tail = 0;   // wave-uniform queue positions (A, and phase 2's)

        // phase 2: residuals, weights, Jacobian rows and accumulation of queue slot `slot`
        auto consume = [&](int slot, bool active) {
          // 27 H / b sums; slots 27..31 only pad the butterfly, whose lanes keep each slot apart, so any value
          // will do there.  rho is summed per lane in FP64 (finite differences of F resolve small changes).
          T v[32];
#pragma unroll
          for (int k = 0; k < 32; ++k) v[k] = k < ACC_F ? T(0) : any_value<T>();
          if (active) {
            const int pix = Q.pix[slot];
            const int cellv = Q.cell[slot];
            const int x0 = cellv & 0xffff, y0 = cellv >> 16;
            const T al = Q.al[slot], be = Q.be[slot];
            const T px = Q.px[slot], py = Q.py[slot], pz = Q.pz[slot];
            const T ed = Q.ed[slot], Gxd = Q.gxd[slot], Gyd = Q.gyd[slot];
            const int corner = (int)__umul24((uint32_t)(y0 - 1), (uint32_t)Wt) + (x0 - 1);
            const T w00 = (T(1) - al) * (T(1) - be), w01 = al * (T(1) - be);
            const T w10 = (T(1) - al) * be, w11 = al * be;
            T Is, ns0 = T(0), ns1 = T(0), ns2 = T(0);
            T Vg, Gxg, Gyg;
            T Vn[3] = {T(0), T(0), T(0)}, Gxn[3] = {T(0), T(0), T(0)}, Gyn[3] = {T(0), T(0), T(0)};
            if (NCH == 5) {
                float4 s4;
                float4 q4[12];
                if (BF) {
                    s4 = ld_bf16x4(r_satt, pix * 8, 0);
                    load_stencil<float4, 8>(q4, [&](int vo, int so) { return ld_bf16x4(r_tatt, vo, so); }, corner * 8,
                                            Wt * 8);
                } else {
                    s4 = ld_f32x4(r_satt, pix * 16, 0);
                    load_stencil<float4, 16>(q4, [&](int vo, int so) { return ld_f32x4(r_tatt, vo, so); }, corner * 16,
                                             Wt * 16);
                }
                Is = s4.x; ns0 = s4.y; ns1 = s4.z; ns2 = s4.w;
                float tI[12], tX[12], tY[12], tZ[12];
#pragma unroll
                for (int k = 0; k < 12; ++k) { tI[k] = q4[k].x; tX[k] = q4[k].y; tY[k] = q4[k].z; tZ[k] = q4[k].w; }
#define SAMPLE(arr, V, GX, GY)                                                                             \
    sample_channel<T, GM>((T)arr[0], (T)arr[1], (T)arr[2], (T)arr[3], (T)arr[4], (T)arr[5], (T)arr[6],      \
                          (T)arr[7], (T)arr[8], (T)arr[9], (T)arr[10], (T)arr[11], w00, w01, w10, w11, al, \
                          be, V, GX, GY)
                SAMPLE(tI, Vg, Gxg, Gyg);
                SAMPLE(tX, Vn[0], Gxn[0], Gyn[0]);
                SAMPLE(tY, Vn[1], Gxn[1], Gyn[1]);
                SAMPLE(tZ, Vn[2], Gxn[2], Gyn[2]);
            } else {
                float tI[12];
                if (BF) {
                    Is = ld_bf16(r_satt, pix * 2, 0);
                    load_stencil<float, 2>(tI, [&](int vo, int so) { return ld_bf16(r_tatt, vo, so); }, corner * 2,
                                           Wt * 2);
                } else {
                    Is = ld_f32(r_satt, pix * 4, 0);
                    load_stencil<float, 4>(tI, [&](int vo, int so) { return ld_f32(r_tatt, vo, so); }, corner * 4,
                                           Wt * 4);
                }
                SAMPLE(tI, Vg, Gxg, Gyg);
#undef SAMPLE
            }
            const T eg = Is - Vg;
            T chi2 = om_g * eg * eg + om_d * ed * ed;
            T en[3] = {T(0), T(0), T(0)}, nr[3] = {T(0), T(0), T(0)};
            if (NCH == 5) {
                // normal cue: the source normal rotated into the target sensor frame
                // rotated in FP64: the rounding of an FP32 rotation would turn every normal of the
                // pair alike
                const double m0 = (double)ns0, m1 = (double)ns1, m2 = (double)ns2;
#pragma unroll
                for (int k = 0; k < 3; ++k) nr[k] = (T)fma(Rd[3 * k], m0, fma(Rd[3 * k + 1], m1, Rd[3 * k + 2] * m2));
#pragma unroll
                for (int k = 0; k < 3; ++k) { en[k] = nr[k] - Vn[k]; chi2 += om_n * en[k] * en[k]; }
            }
            if (DBG) {
                float *rr = a.dbg_res + 5 * (int64_t)pix;
                rr[0] = (float)eg; rr[1] = (float)ed; rr[2] = (float)en[0]; rr[3] = (float)en[1]; rr[4] = (float)en[2];
                a.dbg_status[pix] = 0;
            }
            // Huber on sqrt(chi^2): w = d rho / d chi^2
            T w = T(1), rhov = chi2;
            if (delta > T(0)) {
                // the reciprocal square root only where chi^2 is beyond delta^2 (never of a tiny value)
                if (chi2 > delta * delta) {
                    const T isq = fast_rsq(chi2), sq = chi2 * isq;
                    w = delta * isq;
                    rhov = delta * (T(2) * sq - delta);
                }
            }
            acc_F += (double)rhov;
            n_valid += 1;
            // projective Jacobian rows Pi0 = d u / d p_bar, Pi1 = d v / d p_bar
            T P00, P01, P02, P10, P11, P12, zx, zy, zz;
            if (TM == MODEL_PINHOLE) {
                const T iz = fast_rcp(pz);
                P00 = fx * iz; P01 = T(0); P02 = -fx * px * iz * iz;
                P10 = T(0); P11 = fy * iz; P12 = -fy * py * iz * iz;
                zx = T(0); zy = T(0); zz = T(1);
            } else {
                const T r2 = px * px + py * py, n2 = r2 + pz * pz;
                const T irho = fast_rsq(r2), ir = fast_rsq(n2);
                const T rho = r2 * irho, ir2 = irho * irho, in2 = ir * ir, k1 = pz * irho * in2;
                P00 = -fx * py * ir2; P01 = fx * px * ir2; P02 = T(0);
                P10 = -fy * px * k1; P11 = -fy * py * k1; P12 = fy * rho * in2;
                zx = px * ir; zy = py * ir; zz = pz * ir;
            }
            const T y2x = T(2) * (px + cc[0]), y2y = T(2) * (py + cc[1]), y2z = T(2) * (pz + cc[2]);
            T J[6];
            // a = -(Gx Pi0 + Gy Pi1), leaving out the projective Jacobian's structural zeros (spherical:
            // d u' / d z = 0; pinhole: d u' / d y = d v' / d x = 0)
            auto proj_a = [&](T Gx, T Gy, T &a0, T &a1, T &a2) {
                if (TM == MODEL_PINHOLE) { a0 = -(Gx * P00); a1 = -(Gy * P11); a2 = -(Gx * P02 + Gy * P12); }
                else { a0 = -(Gx * P00 + Gy * P10); a1 = -(Gx * P01 + Gy * P11); a2 = -(Gy * P12); }
            };
            // point-space derivatives a^c = d e^c / d p_bar
            T ag0, ag1, ag2, ad0, ad1, ad2;
            proj_a(Gxg, Gyg, ag0, ag1, ag2);
            proj_a(Gxd, Gyd, ad0, ad1, ad2);
            ad0 += zx; ad1 += zy; ad2 += zz;
            // intensity: a = -(Gx Pi0 + Gy Pi1)
            row_from_a(J, ag0, ag1, ag2, y2x, y2y, y2z);
            if (ADJ) accumulate_row_b(acc_b, J, eg, w * om_g);
            else add_cue_row(v, acc64, J, eg, w * om_g);
            // depth / range: a = d zeta / d p_bar - (Gx Pi0 + Gy Pi1)
            row_from_a(J, ad0, ad1, ad2, y2x, y2y, y2z);
            if (ADJ) accumulate_row_b(acc_b, J, ed, w * om_d);
            else add_cue_row(v, acc64, J, ed, w * om_d);
            if (NCH == 5) {
                // normal rows: image term plus the rotation-only term 2 (e_k x n')
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    T an0, an1, an2;
                    proj_a(Gxn[k], Gyn[k], an0, an1, an2);
                    row_from_a(J, an0, an1, an2, y2x, y2y, y2z);
                    if (k == 0) { J[4] -= T(2) * nr[2]; J[5] += T(2) * nr[1]; }
                    if (k == 1) { J[3] += T(2) * nr[2]; J[5] -= T(2) * nr[0]; }
                    if (k == 2) { J[3] -= T(2) * nr[1]; J[4] += T(2) * nr[0]; }
                    if (ADJ) accumulate_row_b(acc_b, J, en[k], w * om_n);
                    else add_cue_row(v, acc64, J, en[k], w * om_n);
                }
            }
            if (ADJ) {
                // dF/de^c = 2 w Omega^c e^c (times the incoming gradient)
                const T sc = (T)a.adj_scale * T(2) * w;
                const T kg = sc * om_g * eg, kd = sc * om_d * ed;
                const T kn0 = sc * om_n * en[0], kn1 = sc * om_n * en[1], kn2 = sc * om_n * en[2];
                // target: e^c = zeta^c - V^c, V^c bilinear in the 4 taps
                const int64_t toff = kt.off;
                const int base = y0 * Wt + x0;
                const int tap[4] = {base, base + 1, base + Wt, base + Wt + 1};
                const T wt[4] = {w00, w01, w10, w11};
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int64_t o = toff + tap[q];
                    unsafeAtomicAdd(a.g_int + o, (float)(-kg * wt[q]));
                    unsafeAtomicAdd(a.g_dep + o, (float)(-kd * wt[q]));
                    if (NCH == 5) {
                        unsafeAtomicAdd(a.g_nrm + 3 * o, (float)(-kn0 * wt[q]));
                        unsafeAtomicAdd(a.g_nrm + 3 * o + 1, (float)(-kn1 * wt[q]));
                        unsafeAtomicAdd(a.g_nrm + 3 * o + 2, (float)(-kn2 * wt[q]));
                    }
                }
                // source intensity, normal (through R n_u) and depth (through p_bar = R d ray + t)
                const int64_t so = ks.off + pix;
                unsafeAtomicAdd(a.g_int + so, (float)kg);
                int row = (int)__umulhi((uint32_t)pix, magic);
                int col = pix - row * Ws;
                if (col < 0) { row -= 1; col += Ws; }
                const L2 lc = lcol[col], lr = lrow[row];
                T rx, ry, rz;
                if (SM == MODEL_SPHERICAL) { rx = lr.x * lc.x; ry = lr.x * lc.y; rz = lr.y; }
                else { rx = lc.x; ry = lr.x; rz = T(1); }
                const T dp0 = (T)Rd[0] * rx + (T)Rd[1] * ry + (T)Rd[2] * rz;
                const T dp1 = (T)Rd[3] * rx + (T)Rd[4] * ry + (T)Rd[5] * rz;
                const T dp2 = (T)Rd[6] * rx + (T)Rd[7] * ry + (T)Rd[8] * rz;
                T gd = kg * (ag0 * dp0 + ag1 * dp1 + ag2 * dp2) + kd * (ad0 * dp0 + ad1 * dp1 + ad2 * dp2);
                if (NCH == 5) {
                    const T kk[3] = {kn0, kn1, kn2};
#pragma unroll
                    for (int k = 0; k < 3; ++k)
                        gd += kk[k] * (-(Gxn[k] * P00 + Gyn[k] * P10) * dp0 - (Gxn[k] * P01 + Gyn[k] * P11) * dp1 -
                                       (Gxn[k] * P02 + Gyn[k] * P12) * dp2);
#pragma unroll
                    for (int j = 0; j < 3; ++j)
                        unsafeAtomicAdd(a.g_nrm + 3 * so + j,
                                        (float)(kn0 * (T)Rd[j] + kn1 * (T)Rd[3 + j] + kn2 * (T)Rd[6 + j]));
                }
                unsafeAtomicAdd(a.g_dep + so, (float)gd);
            }
          }
          if (!ADJ && F32) acc_hb += (double)wave_reduce_scatter(v, lane);
        };

        // phase 1a: every source pixel of a chunk -- unprojection, transform, a first projection good to a
        // fraction of a pixel, and the depth-interval test; survivors are appended to queue A in pixel order
        // The 12-tap occlusion gate of cell (x0, y0) inside the image: every tap valid and on the surface the
        // point lands on.  Invalid target depths hold a large negative sentinel, so one bound on the largest
        // |D - zeta| also rejects them.  Tested in FP64 in both paths (the taps are exact in FP64): a mask
        // decision does not depend on the evaluation precision.
        auto gate_at = [&](float (&tD)[12], int x0, int y0, double zeta) {
            load_stencil<float, 4>(tD, [&](int vo, int so) { return ld_f32(r_tdep, vo, so); },
                                   ((int)__umul24((uint32_t)(y0 - 1), (uint32_t)Wt) + (x0 - 1)) * 4, Wt * 4);
            float dmin = tD[0], dmax = tD[0];
#pragma unroll
            for (int k = 1; k < 12; ++k) { dmin = fminf(dmin, tD[k]); dmax = fmaxf(dmax, tD[k]); }
            return fmax((double)dmax - zeta, zeta - (double)dmin) <= taud_gate;
        };

        // phase 1b: 64 queued points at a time -- the exact projection and cell, the stencil inside the image,
        // the occlusion gate and the depth channel; valid correspondences are appended to phase 2's queue
        // (Pinhole targets take it in place, for the lanes of a chunk, from phase 1a's registers: their exact
        // projection costs little, so they keep no queue A and no interval test.)
        auto stage_b_core = [&](int pix_in, int kcr, double X, double Y, double Z, bool active) {
            bool valid = false, band = false;
            int pix = any_value<int>(), x0 = any_value<int>(), y0 = any_value<int>();
            T al = any_value<T>(), be = any_value<T>(), px = any_value<T>(), py = any_value<T>();
            T pz = any_value<T>(), edv = any_value<T>(), gxd = any_value<T>(), gyd = any_value<T>();
            if (active) {
                pix = pix_in;
                px = (T)X; py = (T)Y; pz = (T)Z;
                const int kc = kcr & 0x7fff, kr = (kcr >> 16) & 0x7fff;
                const bool near = !DBG || TM == MODEL_PINHOLE || kcr < 0;
                const bool pass = !DBG || TM == MODEL_PINHOLE || (kcr & 0x8000) != 0;
                double u, v, zeta;
                if (TM == MODEL_PINHOLE) {
                    const double iz = rcp_f64(Z);
                    u = fma(st_fx * X, iz, st_cx);
                    v = fma(st_fy * Y, iz, st_cy);
                    zeta = Z;
                } else {
                    // exact angular offset from the table ray the first projection named:
                    // az - az_k = atan2(Y cos az_k - X sin az_k, X cos az_k + Y sin az_k), a small angle, and
                    // likewise for the elevation
                    const double r2 = fma(X, X, Y * Y), n2 = fma(Z, Z, r2);
                    zeta = sqrt_f64(n2);
                    const double rho = sqrt_f64(r2);
                    const double2 cs = ld_f64x2(r_lut, (t_lcol + kc) * 16), rs = ld_f64x2(r_lut, (t_lrow + kr) * 16);
                    const double tu = fma(Y, cs.x, -X * cs.y) * rcp_f64(fma(X, cs.x, Y * cs.y));
                    const double tv = fma(Z, rs.x, -rho * rs.y) * rcp_f64(fma(rho, rs.x, Z * rs.y));
                    u = fma(st_fx, atan_small(tu), (double)kc);
                    v = fma(st_fy, atan_small(tv), (double)kr);
                }
                if (DBG) { a.dbg_status[pix] = 3; a.dbg_uv[pix] = make_float2((float)u, (float)v); }
                // the integer cell floor(u'), and the stencil inside the image
                bool ok = near && u >= 1.0 && u < (double)(Wt - 2) && v >= 1.0 && v < (double)(Ht - 2);
                double du = 0.0, dv = 0.0;
                if (ok) {
                    x0 = (int)u; y0 = (int)v;
                    du = u - (double)x0; dv = v - (double)y0;
                    al = (T)du; be = (T)dv;
                }
                if (ZB && ok && a.zpass) {
                    // z-buffer pass: keep the nearest predicted depth per target cell (depths are positive, so
                    // their FP32 bit patterns order like the values); nothing queued
                    atomicMin(zb + y0 * Wt + x0, __float_as_uint((float)zeta));
                    ok = false;
                }
                if (ok) {
                    if (DBG) { a.dbg_status[pix] = 4; a.dbg_cell[pix] = make_int2(x0, y0); }
                    float tD[12];
                    const bool gate = gate_at(tD, x0, y0, zeta);
                    // boundary band: the coordinate is within kBandPx of a cell boundary, where floor(u') can
                    // differ between exact arithmetic and any rounding of it, and the point passes the gate in
                    // its cell or in a cell across that boundary (otherwise no rounding changes its outcome)
                    const bool bu = fabs(du - 0.5) > 0.5 - kBandPx, bv = fabs(dv - 0.5) > 0.5 - kBandPx;
                    band = (bu || bv) && (DBG || pass) && (ZB ? !a.zpass : true);
                    // (rare: a wave-uniform branch, so the common path carries none of it)
                    if (__builtin_expect(__ballot(band && !gate) != 0, 0)) {
                        if (band && !gate) {
                            bool other = false;
                            const int su = du < 0.5 ? -1 : 1, sv = dv < 0.5 ? -1 : 1;
                            for (int k = 1; k < 4; ++k) {
                                const int cx = x0 + ((k & 1) ? su : 0), cy = y0 + ((k & 2) ? sv : 0);
                                if (((k & 1) && !bu) || ((k & 2) && !bv)) continue;
                                if (cx < 1 || cx > Wt - 3 || cy < 1 || cy > Ht - 3) continue;
                                float tA[12];
                                other = other || gate_at(tA, cx, cy, zeta);
                            }
                            band = other;
                        }
                    }
                    // debug launches: status 5 marks a point the interval test dropped although it passes the
                    // gate in a cell it can reach (never expected; the parity tests check for it)
                    if (DBG && !pass && (gate || band)) a.dbg_status[pix] = 5;
                    band = band && pass;
                    bool vis = gate && pass;
                    // z-buffer variant: also no more than tau behind the nearest of the pair's own points in this
                    // cell (both depths as FP32, compared in FP64)
                    if (ZB && vis)
                        vis = (double)(float)zeta - (double)__uint_as_float(zb[y0 * Wt + x0]) <= taud_gate;
                    if (vis) {
                        const T w00 = (T(1) - al) * (T(1) - be), w01 = al * (T(1) - be);
                        const T w10 = (T(1) - al) * be, w11 = al * be;
                        // e_d = zeta - D(u') taken relative to the tap at (x0, y0): the taps lie within tau of
                        // zeta, so their differences are exact and the large common part cancels in FP64 before
                        // anything is rounded to the evaluation precision; the image Jacobian only takes
                        // differences of taps
                        const float d0 = tD[1];
                        const T Vr = w01 * (T)(tD[2] - d0) + w10 * (T)(tD[5] - d0) + w11 * (T)(tD[6] - d0);
                        sample_grad<T, GM>((T)tD[0], (T)tD[1], (T)tD[2], (T)tD[3], (T)tD[4], (T)tD[5], (T)tD[6],
                                           (T)tD[7], (T)tD[8], (T)tD[9], (T)tD[10], (T)tD[11], w00, w01, w10, w11,
                                           al, be, gxd, gyd);
                        edv = (T)(zeta - (double)d0) - Vr;
                        valid = true;
                    }
                }
            }
            n_band += __popcll(__ballot(band));
            // append the valid lanes to phase 2's queue in lane (= pixel) order
            const uint64_t mask = __ballot(valid);
            if (valid) {
                const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                           __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
                const int slot = (tail + rank) & (kQ - 1);
                Q.pix[slot] = pix;
                Q.cell[slot] = x0 | (y0 << 16);
                Q.al[slot] = al; Q.be[slot] = be;
                Q.px[slot] = px; Q.py[slot] = py; Q.pz[slot] = pz;
                Q.ed[slot] = edv; Q.gxd[slot] = gxd; Q.gyd[slot] = gyd;
            }
            tail += __popcll(mask);
            __builtin_amdgcn_wave_barrier();
        };
        auto stage_b = [&](int slot_a, bool active) {
            int pix = any_value<int>(), kcr = any_value<int>();
            double X = any_value<double>(), Y = any_value<double>(), Z = any_value<double>();
            if (active) {
                pix = QA.pix[slot_a];
                kcr = QA.kcr[slot_a];
                X = QA.X[slot_a]; Y = QA.Y[slot_a]; Z = QA.Z[slot_a];
            }
            stage_b_core(pix, kcr, X, Y, Z, active);
        };

        // A chunk's source depth and ray-table entries, loaded one chunk ahead so that phase 1a finds them in
        // registers (lanes past the item's end read harmless in-buffer values and are discarded)
        struct ChunkLoads {
            float d;
            double2 lc, lr;
        };
        // row and column of the first pixel of the chunk fetched next (rows of 64 or more pixels): split once per
        // item on the scalar unit, then advanced by 64 pixels per chunk (at most one row boundary)
        int f_r0 = (int)__umulhi((uint32_t)px0, magic);
        int f_c0 = px0 - f_r0 * Ws;
        if (f_c0 < 0) { f_r0 -= 1; f_c0 += Ws; }   // the reciprocal can only round up
        auto fetch = [&](int cbase) {
            int row, col;
            if (Ws >= 64) {
                // the chunk's 64 pixels span at most two rows
                col = f_c0 + lane;
                const bool next = col >= Ws;
                row = next ? f_r0 + 1 : f_r0;
                col = next ? col - Ws : col;
                f_c0 += 64;
                if (f_c0 >= Ws) { f_c0 -= Ws; f_r0 += 1; }
            } else {
                const int pix = cbase + lane;
                row = (int)__umulhi((uint32_t)pix, magic);
                col = pix - row * Ws;
                if (col < 0) { row -= 1; col += Ws; }
            }
            ChunkLoads L;
            L.d = ld_f32(r_sdep, (cbase + lane) * 4, 0);
            L.lc = ld_f64x2(r_lut, (s_lcol + col) * 16);
            L.lr = ld_f64x2(r_lut, (s_lrow + row) * 16);
            return L;
        };
        ChunkLoads cur = fetch(px0);

        auto stage_a = [&](int cbase) {
            const int pix = cbase + lane;
            bool keep = false;
            // queued only where kept: elsewhere any value will do (no instructions to clear them)
            int kcr = any_value<int>();
            double X = any_value<double>(), Y = any_value<double>(), Z = any_value<double>();
            const ChunkLoads L = cur;
            // Phase 1a runs on every lane (nearly every source pixel has a depth, so a branch on it skips no
            // chunk; lanes without one are dropped at the end), except where the branch measured faster: the
            // z-buffer variants (whose register allocation fits four waves per SIMD only with it) and the FP64
            // kernels into pinhole targets.  The next chunk's loads, one chunk ahead, go ahead of that branch
            // (never inside it: fetch also advances the next chunk's row and column), elsewhere after the
            // unprojection has its operands.
            constexpr bool kDepthBranch = ZB || (!F32 && TM == MODEL_PINHOLE);
            if (kDepthBranch && cbase + 64 < px1) cur = fetch(cbase + 64);
            const float Ds = pix < px1 ? L.d : 0.f;
            if (DBG && pix < px1) a.dbg_status[pix] = Ds > 0.f ? 2 : 1;
            n_eval += __popcll(__ballot(Ds > 0.f));
            if (!kDepthBranch || Ds > 0.f) {
                // Geometry in FP64 in both paths (on this chip FP64 vector arithmetic issues at the FP32
                // rate): unprojection q = d * ray(u) from the FP64 ray table, p_bar = R q + t, and the
                // predicted depth/range.  Cells, masks and the large-magnitude part of the depth residual then
                // carry no FP32 rounding.
                const double2 lcd = L.lc, lrd = L.lr;
                const double dd = (double)Ds;
                double q0, q1, q2;
                if (SM == MODEL_SPHERICAL) { q0 = dd * (lrd.x * lcd.x); q1 = dd * (lrd.x * lcd.y); q2 = dd * lrd.y; }
                else { q0 = dd * lcd.x; q1 = dd * lrd.x; q2 = dd; }
                if (!kDepthBranch && cbase + 64 < px1) cur = fetch(cbase + 64);
                X = fma(Rd[0], q0, fma(Rd[1], q1, fma(Rd[2], q2, td[0])));
                Y = fma(Rd[3], q0, fma(Rd[4], q1, fma(Rd[5], q2, td[1])));
                Z = fma(Rd[6], q0, fma(Rd[7], q1, fma(Rd[8], q2, td[2])));
                // first projection (Sec. III): pinhole exact; spherical a coarse FP32 estimate (within 0.49 px,
                // checked per sensor on the host), which names the table rays of phase 1b's exact offsets
                bool ok, near;
                float zf, ua, va;   // predicted depth/range in FP32 (within 2e-7 relative) for the interval test
                if (TM == MODEL_PINHOLE) {
                    ok = Z >= st_dmin;
                    near = true;
                    ua = 0.f; va = 0.f; zf = 0.f;
                } else {
                    const double r2 = fma(X, X, Y * Y), n2 = fma(Z, Z, r2);
                    ok = (r2 > 0.0) && (n2 >= st_dmin * st_dmin);
                    const float n2f = (float)n2, r2f = (float)r2, irho = __builtin_amdgcn_rsqf(r2f);
                    zf = n2f * __builtin_amdgcn_rsqf(n2f);
                    ua = (float)st_fx * atan2_coarse((float)Y, (float)X) + (float)st_cx;
                    if (flags & 2) {
                        // every elevation the image can reach is below 45 degrees: atan of tan(el) = Z / rho
                        // by the coarse quadratic, no division; beyond 45 degrees the point is outside
                        const float te = (float)Z * irho;
                        va = fabsf(te) <= 1.f ? fmaf((float)st_fy, atan_unit(te), (float)st_cy) : -2.f;
                    } else {
                        va = (float)st_fy * atan2_coarse((float)Z, r2f * irho) + (float)st_cy;
                    }
                    // far outside the image the estimate decides alone (it is good to a fraction of a pixel);
                    // inside, the nearest table ray is within 1 px, so the offset angle is small
                    near = ua > -1.f && ua < (float)Wt && va > -1.f && va < (float)Ht;
                }
                const int kc = (int)fminf(fmaxf(rintf(ua), 0.f), (float)(Wt - 1));
                const int kr = (int)fminf(fmaxf(rintf(va), 0.f), (float)(Ht - 1));
                // The exact cell is one of {kc - 1, kc} x {kr - 1, kr} (|u' - ua| < 0.5) or outside the cells
                // whose stencil lies inside the image.  The plane holds the range of predicted depths for which
                // one of them can pass the occlusion gate, widened beyond the FP32 error of zf; outside it the gate
                // fails in every one, so a rejected point changes nothing.
                bool pass = true;
                if (flags & 1) {
                    const float2 g = ld_f32x2(r_gate, (int)(__umul24((uint32_t)kr, (uint32_t)Wt) + kc) * 8);
                    pass = zf >= g.x && zf <= g.y;
                }
                // debug launches take every projected point through phase 1b (complete per-pixel statuses) and
                // apply the interval test's verdict at the end
                keep = Ds > 0.f && (DBG ? ok : (ok && near && pass));
                kcr = kc | (kr << 16);
                if (DBG) kcr |= (pass ? 0x8000 : 0) | (near ? (int)0x80000000 : 0);
            }
            if (TM == MODEL_PINHOLE) {   // phase 1b in place
                stage_b_core(pix, kcr, X, Y, Z, keep);
                return;
            }
            const uint64_t mask = __ballot(keep);
            if (keep) {
                const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                           __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
                const int slot = (tailA + rank) & (kQ - 1);
                QA.pix[slot] = pix;
                QA.kcr[slot] = kcr;
                QA.X[slot] = X; QA.Y[slot] = Y; QA.Z[slot] = Z;
            }
            tailA += __popcll(mask);
            __builtin_amdgcn_wave_barrier();
        };

        // The wave's chunks go through phase 1a; each later stage takes 64 queued entries at a time (every lane
        // busy), and after the last chunk the partial remainders (inactive lanes join the butterfly with
        // zeros).  Queue occupancy stays below 128: at most 63 wait before a stage appends at most 64.
        for (int cbase = px0; cbase < px1; cbase += 64) {
            stage_a(cbase);
            if (TM == MODEL_SPHERICAL && tailA - headA >= 64) {
                stage_b((headA + lane) & (kQ - 1), true);
                headA += 64;
                __builtin_amdgcn_wave_barrier();
            }
            if (tail - head >= 64) {
                consume((head + lane) & (kQ - 1), true);
                head += 64;
                __builtin_amdgcn_wave_barrier();
            }
        }
        if (TM == MODEL_SPHERICAL && tailA > headA) {
            stage_b((headA + lane) & (kQ - 1), lane < tailA - headA);
            headA = tailA;
            __builtin_amdgcn_wave_barrier();
        }
        while (tail > head) {   // at most two rounds (up to 126 entries)
            consume((head + lane) & (kQ - 1), lane < tail - head);
            head += min(tail - head, 64);
            __builtin_amdgcn_wave_barrier();
        }

        // the wave's totals (fixed order: deterministic), value k in lane k, one store per item
        double outv = 0.0;
        if (!ADJ && F32) {
            const double t = __shfl(acc_hb, (2 * lane) & 63, 64);   // lanes 2k, 2k + 1 hold sum k
            if (lane < ACC_F) outv = t;
        }
#pragma unroll
        for (int k = ADJ ? ACC_B : (F32 ? ACC_F : 0); k < ACC_USED; ++k) {
            double v = k < ACC_F ? (ADJ ? acc_b[k - ACC_B] : acc64[F32 ? 0 : k])
                                 : (k == ACC_F ? acc_F
                                               : (k == ACC_VALID ? (double)n_valid
                                                                 : (lane == 0 ? (double)(k == ACC_EVAL ? n_eval : n_band)
                                                                              : 0.0)));
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
            if (lane == k) outv = v;
        }
        if (lane < kAcc) static_cast<double *>(a.partials)[(int64_t)item * kAcc + lane] = outv;
    }
}

// Depth-interval plane of one keyframe (one thread per texel (kc, kr)): over the cells (x0, y0) in
// {kc - 1, kc} x {kr - 1, kr} with the stencil inside the image, those whose 12 depth taps span at most
// 2 tau + 1e-6 m (a wider span fails the gate max(dmax - zeta, zeta - dmin) <= tau for every zeta, FP64
// rounding included) give lo = min of their largest taps and hi = max of their smallest taps.  A point
// passing the gate in one of them has dmax - zeta <= tau and zeta - dmin <= tau there, hence, rounding
// being monotone, lo - zeta <= tau and zeta - hi <= tau.
__global__ void gate_plane_kernel(const float *__restrict__ dep, float2 *__restrict__ out, int H, int W, double tau)
{
    const int kc = blockIdx.x * blockDim.x + threadIdx.x, kr = blockIdx.y;
    if (kc >= W) return;
    // the 5 x 5 texels rows kr - 2 .. kr + 2, columns kc - 2 .. kc + 2 hold every tap of the four cells
    float d[5][5];
#pragma unroll
    for (int i = 0; i < 5; ++i)
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            const int y = kr - 2 + i, x = kc - 2 + j;
            d[i][j] = (y >= 0 && y < H && x >= 0 && x < W) ? dep[(int64_t)y * W + x] : kNoDepth;
        }
    float lo = INFINITY, hi = -INFINITY;
#pragma unroll
    for (int dy = -1; dy <= 0; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 0; ++dx) {
            const int x0 = kc + dx, y0 = kr + dy;
            if (x0 < 1 || x0 > W - 3 || y0 < 1 || y0 > H - 3) continue;
            // in d, row y0 of cell (x0, y0) is index dy + 2 and its column x0 index dx + 2
            const int r = dy + 2, c = dx + 2;
            const float t[12] = {d[r][c - 1], d[r][c], d[r][c + 1], d[r][c + 2], d[r + 1][c - 1], d[r + 1][c],
                                 d[r + 1][c + 1], d[r + 1][c + 2], d[r - 1][c], d[r - 1][c + 1], d[r + 2][c],
                                 d[r + 2][c + 1]};
            float mn = t[0], mx = t[0];
#pragma unroll
            for (int k = 1; k < 12; ++k) { mn = fminf(mn, t[k]); mx = fmaxf(mx, t[k]); }
            if ((double)mx - (double)mn > 2.0 * tau + 1e-6) continue;
            lo = fminf(lo, mx);
            hi = fmaxf(hi, mn);
        }
    // Predicted depths zeta that can pass: zeta >= lo - tau and zeta <= hi + tau (up to FP64 rounding).  The
    // evaluation tests an FP32 zf within 2e-7 relative of zeta, so the bounds are widened by 1e-6 relative
    // and 1e-9 m and rounded outwards to FP32.
    float2 r = make_float2(INFINITY, -INFINITY);
    if (lo < INFINITY) {
        const double l = (double)lo - tau, h = (double)hi + tau;
        r.x = __double2float_rd(l - 1e-6 * fabs(l) - 1e-9);
        r.y = __double2float_ru(h + 1e-6 * fabs(h) + 1e-9);
    }
    out[(int64_t)kr * W + kc] = r;
}

void launch_gate_plane(const float *dep, float2 *gate, int H, int W, double tau, hipStream_t st)
{
    hipLaunchKernelGGL(gate_plane_kernel, dim3((W + 127) / 128, H), dim3(128), 0, st, dep, gate, H, W, tau);
}

template <int NCH, int SM, int TM>
static void launch_adj_t(const EvalArgs &a, int item_base, int n_items, int grid, hipStream_t st)
{
    if (a.zbuf)
        hipLaunchKernelGGL((eval_kernel<float, NCH, SM, TM, 1, false, true, true>), dim3(grid), dim3(kBlock), 0, st, a,
                           item_base, n_items);
    else
        hipLaunchKernelGGL((eval_kernel<float, NCH, SM, TM, 1, false, true>), dim3(grid), dim3(kBlock), 0, st, a,
                           item_base, n_items);
}

void launch_eval_adjoint(const EvalArgs &a, int channels, int sm, int tm, int item_base, int n_items, int grid,
                         hipStream_t st)
{
    const int key = (sm << 1) | tm;
    if (channels == 5) {
        switch (key) {
        case 0: launch_adj_t<5, MODEL_PINHOLE, MODEL_PINHOLE>(a, item_base, n_items, grid, st); break;
        case 1: launch_adj_t<5, MODEL_PINHOLE, MODEL_SPHERICAL>(a, item_base, n_items, grid, st); break;
        case 2: launch_adj_t<5, MODEL_SPHERICAL, MODEL_PINHOLE>(a, item_base, n_items, grid, st); break;
        default: launch_adj_t<5, MODEL_SPHERICAL, MODEL_SPHERICAL>(a, item_base, n_items, grid, st); break;
        }
    } else {
        switch (key) {
        case 0: launch_adj_t<2, MODEL_PINHOLE, MODEL_PINHOLE>(a, item_base, n_items, grid, st); break;
        case 1: launch_adj_t<2, MODEL_PINHOLE, MODEL_SPHERICAL>(a, item_base, n_items, grid, st); break;
        case 2: launch_adj_t<2, MODEL_SPHERICAL, MODEL_PINHOLE>(a, item_base, n_items, grid, st); break;
        default: launch_adj_t<2, MODEL_SPHERICAL, MODEL_SPHERICAL>(a, item_base, n_items, grid, st); break;
        }
    }
}

// dF/d delta_k from b_k (= half the gradient with respect to the right perturbation at
// X0 boxplus delta): translation rows R(q) (2 b_t), rotation rows L(q)^T (2 b_q) with
// L(q) = w I + q q^T / w - [q]x, w = sqrt(1 - |q|^2) (quaternion right increment).
__global__ void pose_grad_kernel(const double *__restrict__ b, const float *__restrict__ delta, double scale,
                                 float *__restrict__ grad, int N)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    double qx = delta[6 * k + 3], qy = delta[6 * k + 4], qz = delta[6 * k + 5];
    const double n2 = qx * qx + qy * qy + qz * qz;
    double w;
    if (n2 < 1.0) {
        w = sqrt(1.0 - n2);
    } else {    // the parameterisation normalises (1, q); its derivative is taken at the normalised q
        const double s = 1.0 / sqrt(1.0 + n2);
        w = s; qx *= s; qy *= s; qz *= s;
    }
    const double R[9] = {1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qz * w), 2 * (qx * qz + qy * w),
                         2 * (qx * qy + qz * w), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qx * w),
                         2 * (qx * qz - qy * w), 2 * (qy * qz + qx * w), 1 - 2 * (qx * qx + qy * qy)};
    const double L[9] = {w + qx * qx / w, qx * qy / w + qz, qx * qz / w - qy,
                         qy * qx / w - qz, w + qy * qy / w, qy * qz / w + qx,
                         qz * qx / w + qy, qz * qy / w - qx, w + qz * qz / w};
    const double *bt = b + 6 * (int64_t)k, *bq = bt + 3;
    for (int i = 0; i < 3; ++i) {
        grad[6 * k + i] = (float)(scale * 2.0 * (R[3 * i] * bt[0] + R[3 * i + 1] * bt[1] + R[3 * i + 2] * bt[2]));
        grad[6 * k + 3 + i] = (float)(scale * 2.0 * (L[i] * bq[0] + L[3 + i] * bq[1] + L[6 + i] * bq[2]));
    }
}

void launch_pose_grad(const double *b, const float *delta, double scale, float *grad, int N, hipStream_t st)
{
    hipLaunchKernelGGL(pose_grad_kernel, dim3((N + 127) / 128), dim3(128), 0, st, b, delta, scale, grad, N);
}

__global__ void delta_to_dx_kernel(const float *__restrict__ delta, double *__restrict__ dx, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dx[i] = (double)delta[i];
}

void launch_delta_to_dx(const float *delta, double *dx, int N, hipStream_t st)
{
    hipLaunchKernelGGL(delta_to_dx_kernel, dim3((6 * N + 255) / 256), dim3(256), 0, st, delta, dx, 6 * N);
}

template <typename T, int NCH, int SM, int TM, int GM, bool DBG>
static void launch_eval_t(const EvalArgs &a, int item_base, int n_items, int grid, hipStream_t st)
{
    if constexpr (std::is_same<T, float>::value) {
        if (a.bf16) {
            hipLaunchKernelGGL((eval_kernel<T, NCH, SM, TM, GM, DBG, false, false, true>), dim3(grid), dim3(kBlock), 0,
                               st, a, item_base, n_items);
            return;
        }
    }
    if (a.zbuf)
        hipLaunchKernelGGL((eval_kernel<T, NCH, SM, TM, GM, DBG, false, true>), dim3(grid), dim3(kBlock), 0, st, a,
                           item_base, n_items);
    else
        hipLaunchKernelGGL((eval_kernel<T, NCH, SM, TM, GM, DBG>), dim3(grid), dim3(kBlock), 0, st, a, item_base,
                           n_items);
}

template <typename T, int NCH, int GM, bool DBG>
static void launch_eval_models(const EvalArgs &a, int sm, int tm, int item_base, int n_items, int grid,
                               hipStream_t st)
{
    if (sm == MODEL_PINHOLE && tm == MODEL_PINHOLE)
        launch_eval_t<T, NCH, MODEL_PINHOLE, MODEL_PINHOLE, GM, DBG>(a, item_base, n_items, grid, st);
    else if (sm == MODEL_PINHOLE)
        launch_eval_t<T, NCH, MODEL_PINHOLE, MODEL_SPHERICAL, GM, DBG>(a, item_base, n_items, grid, st);
    else if (tm == MODEL_PINHOLE)
        launch_eval_t<T, NCH, MODEL_SPHERICAL, MODEL_PINHOLE, GM, DBG>(a, item_base, n_items, grid, st);
    else
        launch_eval_t<T, NCH, MODEL_SPHERICAL, MODEL_SPHERICAL, GM, DBG>(a, item_base, n_items, grid, st);
}

template <typename T, bool DBG>
static void launch_eval_cfg(const EvalArgs &a, int channels, int gm, int sm, int tm, int item_base, int n_items,
                            int grid, hipStream_t st)
{
    if (channels == 5) {
        if (gm == 0) launch_eval_models<T, 5, 0, DBG>(a, sm, tm, item_base, n_items, grid, st);
        else launch_eval_models<T, 5, 1, DBG>(a, sm, tm, item_base, n_items, grid, st);
    } else {
        if (gm == 0) launch_eval_models<T, 2, 0, DBG>(a, sm, tm, item_base, n_items, grid, st);
        else launch_eval_models<T, 2, 1, DBG>(a, sm, tm, item_base, n_items, grid, st);
    }
}

void launch_eval(const EvalArgs &a, int precision, int channels, int grad_mode, int src_model, int tgt_model,
                 bool debug, int item_base, int n_items, int grid, hipStream_t st)
{
    if (precision == 1) {
        if (debug) launch_eval_cfg<double, true>(a, channels, grad_mode, src_model, tgt_model, item_base, n_items, grid, st);
        else launch_eval_cfg<double, false>(a, channels, grad_mode, src_model, tgt_model, item_base, n_items, grid, st);
    } else {
        if (debug) launch_eval_cfg<float, true>(a, channels, grad_mode, src_model, tgt_model, item_base, n_items, grid, st);
        else launch_eval_cfg<float, false>(a, channels, grad_mode, src_model, tgt_model, item_base, n_items, grid, st);
    }
}

// ------------------------------------------------------------------ per-pair reduction and expansion (FP64)

// One wave per pair: sums the pair's FP64 item partials in item order, then expands S, beta
// into the 12x12 / 12 blocks over [dx_s; dx_t]:
//   H_tt = D^T S D, H_ss = E^T S E, H_st = E^T S D, H_ts = D^T S E, b_t = D^T beta, b_s = E^T beta
// with D = blockdiag(R_ot^T, R_ot^T) and E = D A.
__global__ void __launch_bounds__(64) reduce_pairs_kernel(const double *__restrict__ partials,
                                                          const int32_t *__restrict__ pitems,
                                                          const int32_t *__restrict__ ibeg,
                                                          const int32_t *__restrict__ icnt,
                                                          const PairDev *__restrict__ pairs,
                                                          double *__restrict__ out, int P)
{
    const int p = blockIdx.x;
    const int lane = threadIdx.x;
    __shared__ double sums[kAcc];
    __shared__ double S[36], beta[6], Dm[36], Em[36], SD[36], SE[36];
    if (lane < kAcc) {
        double s = 0.0;
        const int b = ibeg[p], n = icnt[p];
        for (int i = 0; i < n; ++i) s += partials[(int64_t)pitems[b + i] * kAcc + lane];
        sums[lane] = s;
    }
    __syncthreads();
    const PairDev &pd = pairs[p];
    if (lane < 36) {
        const int i = lane / 6, j = lane % 6;
        const int a = i < j ? i : j, c = i < j ? j : i;
        // upper-triangular index of (a, c)
        const int idx = a * 6 - a * (a - 1) / 2 + (c - a);
        S[lane] = sums[ACC_H + idx];
        // D = blockdiag(R_ot^T, R_ot^T)
        double dv = 0.0;
        if ((i < 3) == (j < 3)) dv = pd.D[3 * (i % 3) + (j % 3)];
        Dm[lane] = dv;
        Em[lane] = pd.E[lane];
    }
    if (lane < 6) beta[lane] = sums[ACC_B + lane];
    __syncthreads();
    if (lane < 36) {
        const int i = lane / 6, j = lane % 6;
        double sd = 0.0, se = 0.0;
        for (int k = 0; k < 6; ++k) { sd += S[6 * i + k] * Dm[6 * k + j]; se += S[6 * i + k] * Em[6 * k + j]; }
        SD[lane] = sd;
        SE[lane] = se;
    }
    __syncthreads();
    // symmetric by construction: each mirrored pair of entries is computed once
    double *o = out + (int64_t)p * kPairOut;
    if (lane < 36) {
        const int i = lane / 6, j = lane % 6;
        double st = 0;
        for (int k = 0; k < 6; ++k) st += Em[6 * k + i] * SD[6 * k + j];
        o[12 * i + 6 + j] = st;                 // H_st
        o[12 * (6 + j) + i] = st;               // H_ts = H_st^T
        if (i <= j) {
            double ss = 0, tt = 0;
            for (int k = 0; k < 6; ++k) {
                ss += Em[6 * k + i] * SE[6 * k + j];
                tt += Dm[6 * k + i] * SD[6 * k + j];
            }
            o[12 * i + j] = ss;
            o[12 * j + i] = ss;
            o[12 * (6 + i) + 6 + j] = tt;
            o[12 * (6 + j) + 6 + i] = tt;
        }
    }
    if (lane < 6) {
        double bs = 0, bt = 0;
        for (int k = 0; k < 6; ++k) { bs += Em[6 * k + lane] * beta[k]; bt += Dm[6 * k + lane] * beta[k]; }
        o[144 + lane] = bs;
        o[150 + lane] = bt;
    }
    if (lane == 0) {
        o[156] = sums[ACC_F];
        o[157] = sums[ACC_EVAL];
        o[158] = sums[ACC_VALID];
        o[159] = sums[ACC_BAND];
    }
}

void launch_reduce_pairs(const void *partials, int precision, const int32_t *pitems, const int32_t *ibeg,
                         const int32_t *icnt, const PairDev *pairs, double *pair_out, int P, hipStream_t st)
{
    (void)precision;
    if (P <= 0) return;
    hipLaunchKernelGGL(reduce_pairs_kernel, dim3(P), dim3(64), 0, st, static_cast<const double *>(partials), pitems,
                       ibeg, icnt, pairs, pair_out, P);
}

// ------------------------------------------------------------------ assembly of the 6N x 6N system

__global__ void fill_kernel(double *p, int64_t n, double v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

void launch_fill(double *p, int64_t n, double v, hipStream_t st)
{
    if (n <= 0) return;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(256), 0, st, p, n, v);
}

// One workgroup per nonzero 6x6 block: sums its contributions in pair order.
// blk_ent[k] = 4 * pair + quadrant (0 ss, 1 st, 2 ts, 3 tt).
__global__ void __launch_bounds__(64) assemble_H_kernel(const double *__restrict__ pair_out,
                                                        const int2 *__restrict__ blk_rc,
                                                        const int32_t *__restrict__ blk_ptr,
                                                        const int32_t *__restrict__ blk_ent, int n,
                                                        double *__restrict__ H)
{
    const int blk = blockIdx.x;
    const int lane = threadIdx.x;
    if (lane >= 36) return;
    const int i = lane / 6, j = lane % 6;
    double s = 0.0;
    for (int k = blk_ptr[blk]; k < blk_ptr[blk + 1]; ++k) {
        const int e = blk_ent[k];
        const int p = e >> 2, q = e & 3;
        const int ro = (q >> 1) * 6, co = (q & 1) * 6;
        s += pair_out[(int64_t)p * kPairOut + 12 * (ro + i) + co + j];
    }
    const int2 rc = blk_rc[blk];
    H[(int64_t)(6 * rc.x + i) * n + 6 * rc.y + j] = s;
}

// b per pose variable (bk_ent = 2 * pair + side, side 0 = source, 1 = target), one thread per
// entry of b in the workgroups before the last, and the totals F, evaluated, valid (and the
// boundary-band count) summed over pairs in the last workgroup; every sum runs in a fixed order.
__global__ void __launch_bounds__(256) assemble_b_kernel(const double *__restrict__ pair_out, int P,
                                                         const int32_t *__restrict__ bk_ptr,
                                                         const int32_t *__restrict__ bk_ent, int N,
                                                         double *__restrict__ b, double *__restrict__ totals)
{
    const int tid = threadIdx.x;
    if (blockIdx.x + 1 < gridDim.x) {
        const int r = blockIdx.x * blockDim.x + tid;
        if (r >= 6 * N) return;
        const int k = r / 6, j = r % 6;
        double s = 0.0;
#pragma unroll 4
        for (int e = bk_ptr[k]; e < bk_ptr[k + 1]; ++e) {
            const int ent = bk_ent[e];
            s += pair_out[(int64_t)(ent >> 1) * kPairOut + 144 + 6 * (ent & 1) + j];
        }
        b[r] = s;
        return;
    }
    __shared__ double red[4][256];
    double acc[4] = {0, 0, 0, 0};
#pragma unroll 4
    for (int p = tid; p < P; p += blockDim.x)
        for (int k = 0; k < 4; ++k) acc[k] += pair_out[(int64_t)p * kPairOut + 156 + k];
    for (int k = 0; k < 4; ++k) red[k][tid] = acc[k];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w)
            for (int k = 0; k < 4; ++k) red[k][tid] += red[k][tid + w];
        __syncthreads();
    }
    if (tid < 4) totals[tid] = red[tid][0];
}

void launch_assemble(const double *pair_out, int P, const int2 *blk_rc, const int32_t *blk_ptr,
                     const int32_t *blk_ent, int nblk, const int32_t *bk_ptr, const int32_t *bk_ent, int N,
                     double *H, double *b, double *totals, hipStream_t st)
{
    const int n = 6 * N;
    launch_fill(H, (int64_t)n * n, 0.0, st);
    if (nblk > 0)
        hipLaunchKernelGGL(assemble_H_kernel, dim3(nblk), dim3(64), 0, st, pair_out, blk_rc, blk_ptr, blk_ent, n, H);
    hipLaunchKernelGGL(assemble_b_kernel, dim3((6 * N + 255) / 256 + 1), dim3(256), 0, st, pair_out, P, bk_ptr, bk_ent,
                       N, b, totals);
}

void launch_copy(double *dst, const double *src, int64_t n, hipStream_t st);

}  // namespace pba
