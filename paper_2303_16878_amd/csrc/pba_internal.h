// Internal declarations shared by the HIP sources of libpba (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <utility>
#include <vector>

namespace pba {

constexpr int kBlock = 256;      // threads per evaluation workgroup (4 wave64)
constexpr int kAcc = 32;         // accumulator slots per work item
// accumulator layout: 21 upper-triangular H terms, 6 b terms, F, valid, evaluated, boundary band
enum { ACC_H = 0, ACC_B = 21, ACC_F = 27, ACC_VALID = 28, ACC_EVAL = 29, ACC_BAND = 30, ACC_USED = 31 };
// boundary band: a correspondence whose projected coordinate lies within this many pixels of a
// cell boundary (either coordinate), where the integer cell -- and so the mask -- is decided
constexpr double kBandPx = 1e-4;
constexpr int kPairOut = 160;    // PBA_PAIR_OUT_LEN
// one row of the LM log per iteration: F, lambda, step norm, valid, accepted, solve failed, then
// device wall-clock stamps: evaluation begin / end, iteration begin / end
constexpr int kLogRow = 10;
// packed depth of a pixel without a valid measurement: negative, so it fails any depth test
// and every occlusion bound |D - zeta| <= tau
constexpr float kNoDepth = -1e30f;
constexpr int kXcd = 8;          // work queues per launch: one per accelerator complex die (XCD)
constexpr int kCtrStride = 32;   // queue counters 128 bytes apart: one L2 line each, no shared-line contention
enum { MODEL_PINHOLE = 0, MODEL_SPHERICAL = 1 };

// BF16 storage of the intensity / normal planes: round to nearest even (finite values), and back.
__device__ __forceinline__ uint16_t f32_to_bf16(float f)
{
    const uint32_t b = __float_as_uint(f);
    return (uint16_t)((b + 0x7FFFu + ((b >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint32_t h) { return __uint_as_float(h << 16); }

// Attribute texel k of a plane: 5 cues {I, nx, ny, nz} as float4 or, with BF16 storage, ushort4;
// 2 cues: I as float or uint16.
__device__ __forceinline__ float4 att_get4(const void *p, int bf, int64_t k)
{
    if (!bf) return static_cast<const float4 *>(p)[k];
    const ushort4 h = static_cast<const ushort4 *>(p)[k];
    return make_float4(bf16_to_f32(h.x), bf16_to_f32(h.y), bf16_to_f32(h.z), bf16_to_f32(h.w));
}
__device__ __forceinline__ void att_put4(void *p, int bf, int64_t k, float4 v)
{
    if (!bf) { static_cast<float4 *>(p)[k] = v; return; }
    static_cast<ushort4 *>(p)[k] = make_ushort4(f32_to_bf16(v.x), f32_to_bf16(v.y), f32_to_bf16(v.z), f32_to_bf16(v.w));
}
__device__ __forceinline__ float att_get1(const void *p, int bf, int64_t k)
{
    return bf ? bf16_to_f32(static_cast<const uint16_t *>(p)[k]) : static_cast<const float *>(p)[k];
}
__device__ __forceinline__ void att_put1(void *p, int bf, int64_t k, float v)
{
    if (bf) static_cast<uint16_t *>(p)[k] = f32_to_bf16(v);
    else static_cast<float *>(p)[k] = v;
}

struct SensorDev {
    int32_t model, H, W, npx;
    uint32_t magic_w;            // ceil(2^32 / W): row = umulhi(pix, magic_w) for pix < 2^32 / W
    int32_t early;               // as a target: the evaluation's first projection is within half a pixel of
                                 // the exact one, so the depth-interval plane may reject points early
    int32_t el45;                // spherical: every elevation of the image is below 45 degrees
    double fxd, fyd, cxd, cyd, dmind, dmaxd, taud;
    double Ro[9], to[3];         // sensor -> platform
    int64_t lut_col, lut_row;    // element offsets into the ray tables
};

struct KfDev {
    int32_t sensor, H, W;
    int32_t pose;                // pose variable (keyframes of one rig frame share one)
    int64_t off;                 // texel offset of this keyframe in the image arenas
};

// Per-pair transform from the source sensor frame to the target sensor frame,
// p_bar = Rd q + td for q = pi_s^-1(u, d) (FP64 in both paths), and c = R_ot^T t_ot so that the
// target platform point expressed in the target sensor axes is y'' = p_bar + c.
struct alignas(16) PairDev {
    float c[3], pad;
    double Rd[9], td[3];
    double D[9];                 // R_ot^T: target-sensor axes of the platform perturbation
    double E[36];                // D A: source-pose rows follow as J_s = J' E (6x6 row-major)
    int32_t src, tgt, pad2[2];
};

struct EvalArgs {
    const SensorDev *sensors;
    const KfDev *kfs;
    const PairDev *pairs;
    const float *dep;            // depth plane (pixels without a valid depth hold kNoDepth)
    const float4 *att4;          // 5 channels: {intensity, nx, ny, nz}
    const float *att1;           // 2 channels: intensity
    const ushort4 *att4h;        // the same planes with BF16 storage
    const uint16_t *att1h;
    const float2 *lut32;         // ray tables, FP32
    const double2 *lut64;        // ray tables, FP64
    const float2 *gate;          // depth-interval plane (launch_gate_plane), laid out like dep
    const int32_t *item_pair;
    const int32_t *item_px0;
    const int32_t *item_map;     // nullable: item = item_map[position] (per-pair launches)
    int32_t items_px;
    int32_t lut64_bytes;         // size of the FP64 ray tables (bounds of their buffer loads)
    uint32_t *counter;           // kXcd queue counters of this launch, kCtrStride apart
    void *partials;              // double[n_items][kAcc]
    double omega_g, omega_d, omega_n, huber;
    // loss adjoint outputs (adjoint launches only): arenas laid out like the images
    float *g_int, *g_dep, *g_nrm;
    double adj_scale;
    // z-buffer occlusion variant (nullptr: off): per pair, Ht * Wt FP32 depth bits at zbuf + zoff[pair];
    // zpass = 1 fills it (atomic minimum per cell) instead of evaluating
    uint32_t *zbuf;
    const int64_t *zoff;
    int32_t zpass;
    int32_t bf16;                // intensity / normal planes in BF16 (att4h, att1h)
    // per-pixel inspection outputs (debug launches only)
    uint8_t *dbg_status;
    float2 *dbg_uv;
    int2 *dbg_cell;
    float *dbg_res;
};

// ---- launch wrappers (eval.hip)
void launch_pair_setup(const double *poses, const int2 *pairs, int P, const SensorDev *sensors,
                       const KfDev *kfs, PairDev *out, uint32_t *counters, int ncounters, hipStream_t st);
void launch_eval(const EvalArgs &a, int precision, int channels, int grad_mode, int src_model, int tgt_model,
                 bool debug, int item_base, int n_items, int grid, hipStream_t st);
void launch_eval_adjoint(const EvalArgs &a, int channels, int src_model, int tgt_model, int item_base, int n_items,
                         int grid, hipStream_t st);
void launch_pose_grad(const double *b, const float *delta, double scale, float *grad, int N, hipStream_t st);
void launch_delta_to_dx(const float *delta, double *dx, int N, hipStream_t st);
void launch_reduce_pairs(const void *partials, int precision, const int32_t *pair_items,
                         const int32_t *pair_item_begin, const int32_t *pair_item_count, const PairDev *pairs,
                         double *pair_out, int P, hipStream_t st);
void launch_assemble(const double *pair_out, int P, const int2 *blk_rc, const int32_t *blk_ptr,
                     const int32_t *blk_ent, int nblk, const int32_t *bk_ptr, const int32_t *bk_ent, int N,
                     double *H, double *b, double *totals, hipStream_t st);
void launch_fill(double *p, int64_t n, double v, hipStream_t st);

// ---- launch wrappers (solve.hip)
struct LmState {
    double lam, F_cur, F_cand, step_norm;
    int64_t valid_cur, valid_cand;
    int32_t fail, accepted, use_lm, iter;
};
void launch_damp_copy(const double *H, const double *b, double *A, double *rhs, int n, int anchor,
                      const LmState *lm, double lam_override, hipStream_t st);
struct CholPlan;
// The same into the plan's nested-dissection order (plan.n rows, pattern tiles only); also
// clears *fail.
void launch_damp_copy_perm(const double *H, const double *b, double *A, double *rhs, int n0, int anchor,
                           const LmState *lm, double lam_override, const CholPlan &plan, int32_t *fail,
                           hipStream_t st);
// Tiles of the Cholesky factor that can be nonzero (host-built from the pair graph with the
// factorisation's symbolic fill): for block column k, rcnt[k] tile rows i > k at rows + rbeg[k]
// (device, ascending); for block row k, ccnt[k] tile columns j < k at cols + cbeg[k] (device).
// meta holds rbeg, rcnt, cbeg, ccnt on the device (nblk ints each, in that order), then for each
// block column its first kCholPre tile rows and for each block row its first kCholPre tile
// columns (-1 where there are fewer).
// The panel, trailing update and triangular solves touch only these tiles.
constexpr int kCholPre = 4;
struct CholPlan {
    const int32_t *rows = nullptr, *cols = nullptr, *meta = nullptr;
    std::vector<int> rbeg, rcnt, cbeg, ccnt;
    int np = -1;      // pose variables the plan was built for
    int n = 0;        // order of the factored system (6 NP, or more with nested dissection)
    // Nested-dissection order (nd): the factor works on a permuted system whose dissection blocks
    // are padded to 64-row boundaries, and the factorisation and solves run one elimination-tree
    // level per launch.  Device arrays:
    bool nd = false;
    const int32_t *perm = nullptr;      // n: the 6 NP-system index of each factor row, -1 = padding
    const int32_t *pose_off = nullptr;  // NP: first factor row of each pose variable
    const int32_t *dtiles = nullptr;    // 2 ndt: (tile row, tile column) of the lower tiles of the pattern
    int ndt = 0;
    const int32_t *lcols = nullptr;     // block columns grouped by level: level l at lcols + lbeg[l]
    std::vector<int> lbeg, lcnt;
    const int32_t *tasks = nullptr;     // update tasks, 4 ints each: target tile (a, b), first
    const int32_t *contrib = nullptr;   //   contributing column in contrib, count (ascending columns)
    std::vector<int> tbeg, tcnt;        // level l's tasks at tasks + 4 tbeg[l]
};

// Block pattern of the factor of an n x n system with pose variable v at rows pos[v] .. pos[v] + 5,
// coupled along `edges` (pose-variable pairs): for each 64-wide block column k its tile rows
// below the diagonal (ascending, symbolic fill included) and for each block row its tile columns
// left of the diagonal, and each column's level in the elimination tree (0 = no predecessor).
struct TilePattern {
    int n = 0, nt = 0, nlev = 0;
    std::vector<std::vector<int>> rows, cols;
    std::vector<int> level;
};
TilePattern tile_pattern(int n, const std::vector<int> &pos, const std::vector<std::pair<int, int>> &edges);
// Nested-dissection blocks of the pose graph (nv vertices): leaves of at most `leaf` vertices and
// separators, each block's vertices ascending, every separator after the two parts it separates.
std::vector<std::vector<int>> nd_blocks(int nv, const std::vector<std::pair<int, int>> &edges, int leaf);
// First row of each vertex with the blocks laid out in order, each padded to a multiple of 64 rows;
// n_pad receives the padded order.
std::vector<int> nd_positions(int nv, const std::vector<std::vector<int>> &blocks, int &n_pad);
// The level-scheduled factorisation's lists for a pattern in a nested-dissection order (the
// CholPlan fields of the same names, host side): perm, dtiles, lcols / lbeg / lcnt, and tasks /
// contrib / tbeg / tcnt.
struct NdArrays {
    std::vector<int32_t> perm, dtiles, lcols, tasks, contrib;
    std::vector<int> lbeg, lcnt, tbeg, tcnt;
};
NdArrays nd_arrays(const TilePattern &tp, const std::vector<int> &pos);
// A (n x n, lower triangle used) is overwritten; the factor's panel tiles go to L and, transposed,
// to LT (n x n each), the inverted diagonal blocks W and their transposes to Winv (2 nblk blocks of
// 64 x 64: all W, then all W^T).
// With a nested-dissection plan and x (the right-hand side, factor order), the forward substitution
// runs with the factorisation and x ends up holding y with L y = rhs (launch_chol_solve then runs
// only the backward sweeps); x is ignored in the natural order.
void launch_cholesky(double *A, double *L, double *LT, int n, double *Winv, const CholPlan &plan, int32_t *fail,
                     hipStream_t st, double *x);
// Depth-interval plane of one keyframe (H x W depth plane `dep`, occlusion bound tau): texel (kc, kr)
// holds, over the cells (x0, y0) in {kc - 1, kc} x {kr - 1, kr} whose stencil lies inside the image and
// whose 12 depth taps span at most 2 tau (+1e-6 m), with lo = the smallest of their largest taps and
// hi = the largest of their smallest taps, the predicted-depth range [lo - tau, hi + tau] widened by
// 1e-6 relative and 1e-9 m and rounded outwards to FP32 (+inf / -inf where there is no such cell).
void launch_gate_plane(const float *dep, float2 *gate, int H, int W, double tau, hipStream_t st);
// att / att2: the attribute plane of one keyframe (att_get4 / att_get1 layout, `five` cues or one,
// `bf` BF16 storage)
void launch_downsample(const float *dep, const void *att, int five, int bf, int H, int W, float *dep2, void *att2,
                       int H2, int W2, double tau, hipStream_t st);
void launch_unpack(const float *dep, const void *att, int five, int bf, int npx, float *I, float *D, float *N,
                   hipStream_t st);
void launch_normals(const float *dep, void *att4, int bf, int H, int W, const double2 *lcol, const double2 *lrow,
                    int spherical, double scale, double min_px, double max_px, double tau, int min_count,
                    hipStream_t st);
// Solves L L^T x = x in place with the factor as launch_cholesky leaves it (nested dissection: x
// holds y from launch_cholesky, and only L^T x = y remains).
void launch_chol_solve(const double *L, const double *LT, double *Winv, double *x, int n, const CholPlan &plan,
                       const int32_t *fail, hipStream_t st);
// off: first element of each pose variable's 6 in dx (nested-dissection layout), nullptr = 6 k.
void launch_boxplus(const double *X, const double *dx, const int32_t *off, double *Xout, int N, const int32_t *fail,
                    LmState *lm, hipStream_t st);
void launch_gather_step(double *dst, const double *src, const int32_t *off, int N, hipStream_t st);
void launch_stamp(const LmState *lm, double *logbuf, int log_cap, int which, hipStream_t st);
void launch_lm_decide(LmState *lm, const double *totals_cand, int64_t nH, double *H_cur, const double *H_cand,
                      double *b_cur, const double *b_cand, double *X_cur, const double *X_cand, int N,
                      double *totals_cur, double *logbuf, int log_cap, hipStream_t st);
void launch_copy(double *dst, const double *src, int64_t n, hipStream_t st);

}  // namespace pba
