// libpba runtime: context, buffers, work queue, and the C-ABI entry points of include/pba.h.
// The host only validates, marshals and orders launches; all arithmetic of the
// evaluation, reduction, assembly, solve and update runs in the kernels of eval.hip
// and solve.hip.

#include "pba.h"
#include "pba_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

using namespace pba;

// Working memory of pba_evaluate_noalloc: a fixed array in every GPU's copy of this library's code
// object, held until the process ends.  Host code never passes its name to a kernel (on the host it
// is only a stand-in for the symbol): the device address comes from hipGetSymbolAddress, once per
// device at context creation, and is kept in g_scratch_ptr.
constexpr size_t kScratchBytes = PBA_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    const pba_config *via = nullptr;   // config whose allocator callbacks own p (nullptr: hipMalloc)
};

}  // namespace

// One resolution level of every keyframe: the level's sensors (intrinsics), ray tables, keyframe
// layout and packed image planes.  Level 0 holds the loaded images; level l + 1 is the 2x2
// reduction of level l.
struct ImageSet {
    std::vector<pba_sensor> sensors;
    std::vector<SensorDev> sensors_dev_h;
    std::vector<KfDev> kfs_h;
    int64_t texels = 0;
    DevBuf sensors_d, kfs_d, dep, att4, att1, lut32, lut64;
    DevBuf gate;   // depth-interval plane (launch_gate_plane), one float2 per texel
};

struct pba_ctx {
    pba_config cfg;
    hipStream_t stream = nullptr;
    int num_cu = 256;
    std::string err;

    std::vector<pba_sensor> sensors;   // as registered (level 0)
    std::vector<ImageSet> lv = std::vector<ImageSet>(1);
    int level = 0;                     // the level evaluate / iterate / loss work on
    ImageSet &L() { return lv[level]; }
    std::vector<int32_t> src_h, tgt_h; // the pairs as set
    int N = 0, P = 0;
    int NP = 0;                       // pose variables (N unless keyframes share rig poses)
    std::vector<int32_t> pose_of;     // keyframe -> pose variable; empty: one per keyframe
    bool poses_set = false;
    bool system_valid = false;   // H, b, totals[0..3] hold the system at the current poses
    double lam_carry = -1.0;     // LM damping left by the previous pba_iterate call

    // items
    int items_px = 4096;    // source pixels per work item (one wave's)
    int n_items = 0;
    struct Group { int sm, tm, base, count; };
    std::vector<Group> groups;
    std::vector<int32_t> pair_item_begin, pair_item_count;
    int nblk = 0;

    // device buffers
    DevBuf poses, poses_cand, pairs_d, pair_dev, item_pair, item_px0, pitems, ibeg, icnt, counters, partials, pair_out;
    DevBuf blk_rc, blk_ptr, blk_ent, bk_ptr, bk_ent;
    DevBuf chol_rows, chol_cols, chol_meta;
    DevBuf nd_perm, nd_off, nd_dtiles, nd_lcols, nd_tasks, nd_contrib, dx_nat;
    CholPlan chol;   // tiles of the Cholesky factor that can be nonzero
    DevBuf zbuf, zoff;   // z-buffer occlusion variant: per pair, one FP32 depth per target pixel
    int64_t zcells = 0;
    DevBuf H, b, H_cand, b_cand, totals, A, Winv, dx, lm, fail, logbuf;
    DevBuf dbg_status, dbg_uv, dbg_cell, dbg_res;
    DevBuf loss_delta, loss_poses, g_int, g_dep, g_nrm, g_pose;
    bool loss_ready = false;

    // one captured LM iteration (replayed by pba_iterate)
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    bool graph_valid = false;
    int log_cap = 0;

    // timing
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double eval_ms = 0.0, iterate_ms = 0.0, iter_eval_ms = 0.0;
    int64_t iter_evals = 0;
    double wall_khz = 0.0;   // device wall-clock rate
    int64_t eval_launches = 0, iterations = 0;
    int grid = 0;
};

namespace {

pba_status fail(pba_ctx *c, pba_status s, const char *fmt, ...) __attribute__((format(printf, 3, 4)));
pba_status fail(pba_ctx *c, pba_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return s;
}

#define HIP_OK(expr)                                                                                     \
    do {                                                                                                 \
        hipError_t e_ = (expr);                                                                          \
        if (e_ != hipSuccess) return fail(c, PBA_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));       \
    } while (0)

void release(DevBuf &b)
{
    if (b.p) {
        if (b.via) b.via->dev_free(b.p, b.bytes, b.via->alloc_user);
        else (void)hipFree(b.p);
    }
    b.p = nullptr;
    b.bytes = 0;
    b.via = nullptr;
}

// Device memory of at least `bytes` in b (kept if already large enough), through the caller's
// allocator callbacks when the config has them, else hipMalloc.
pba_status ensure(pba_ctx *c, DevBuf &b, size_t bytes)
{
    if (bytes == 0) bytes = 16;
    if (b.bytes >= bytes) return PBA_OK;
    release(b);
    if (c->cfg.dev_alloc) {
        b.p = c->cfg.dev_alloc(bytes, c->cfg.alloc_user);
        if (!b.p) return fail(c, PBA_ENOMEM, "allocator callback returned NULL for %zu bytes", bytes);
        b.via = &c->cfg;
    } else {
        hipError_t e = hipMalloc(&b.p, bytes);
        if (e != hipSuccess) {
            b.p = nullptr;
            return fail(c, PBA_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
        }
    }
    b.bytes = bytes;
    return PBA_OK;
}

template <typename T>
T *P_(DevBuf &b) { return static_cast<T *>(b.p); }

pba_status upload(pba_ctx *c, DevBuf &b, const void *src, size_t bytes)
{
    pba_status s = ensure(c, b, bytes);
    if (s) return s;
    if (bytes) HIP_OK(hipMemcpyAsync(b.p, src, bytes, hipMemcpyHostToDevice, c->stream));
    return PBA_OK;
}

bool pose_ok(const double *x)
{
    for (int i = 0; i < 12; ++i)
        if (!std::isfinite(x[i])) return false;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += x[3 * k + i] * x[3 * k + j];
            if (std::fabs(s - (i == j ? 1.0 : 0.0)) > 1e-6) return false;
        }
    return true;
}

int n_sys(const pba_ctx *c) { return 6 * c->NP; }
int pose_var(const pba_ctx *c, int kf) { return c->pose_of.empty() ? kf : c->pose_of[kf]; }

// texel preparation: sanitise depth (invalid -> 0; the depth test is made in FP64, as the
// sensor's limits are given) and split into the depth plane and the attribute plane
__global__ void pack_kernel(const float *__restrict__ I, const float *__restrict__ D, const float *__restrict__ Nn,
                            float *__restrict__ dep, void *__restrict__ att, int five, int bf, int npx, double dmin,
                            double dmax)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < npx; i += gridDim.x * blockDim.x) {
        const float d = D[i];
        const bool ok = isfinite(d) && d > 0.f && (double)d >= dmin && (double)d <= dmax;
        const float in = I[i];
        dep[i] = ok ? d : kNoDepth;
        if (five) {
            const float n0 = Nn[3 * (int64_t)i], n1 = Nn[3 * (int64_t)i + 1], n2 = Nn[3 * (int64_t)i + 2];
            att_put4(att, bf, i, ok ? make_float4(in, n0, n1, n2) : make_float4(0.f, 0.f, 0.f, 0.f));
        } else {
            att_put1(att, bf, i, ok ? in : 0.f);
        }
    }
}

// The attribute plane of a level (5 cues: att4, 2 cues: att1; element size per the storage).
void *att_plane(pba_ctx *c, ImageSet &is);
size_t att_bytes(const pba_ctx *c);

void release_images(ImageSet &is)
{
    DevBuf *bufs[] = {&is.sensors_d, &is.kfs_d, &is.dep, &is.att4, &is.att1, &is.lut32, &is.lut64, &is.gate};
    for (DevBuf *b : bufs) release(*b);
}

// Device form of the sensors of one level and their ray tables (FP32 and FP64): per column
// (cos az, sin az) or ((u - cx) / fx, 0), per row (cos el, sin el) or ((v - cy) / fy, 0).
pba_status sensor_tables(pba_ctx *c, ImageSet &is)
{
    std::vector<SensorDev> sd(is.sensors.size());
    std::vector<float2> l32;
    std::vector<double2> l64;
    for (size_t i = 0; i < is.sensors.size(); ++i) {
        const pba_sensor &S = is.sensors[i];
        SensorDev &d = sd[i];
        d.model = S.model; d.H = S.height; d.W = S.width; d.npx = S.height * S.width;
        d.magic_w = (uint32_t)(((1ull << 32) + S.width - 1) / S.width);
        d.fxd = S.fx; d.fyd = S.fy; d.cxd = S.cx; d.cyd = S.cy; d.dmind = S.min_depth; d.dmaxd = S.max_depth;
        d.taud = S.model == PBA_PINHOLE ? c->cfg.occlusion_tau_pinhole : c->cfg.occlusion_tau_spherical;
        // As a target, the evaluation's first projection must lie within half a pixel of the exact one
        // for the depth-interval rejection.  Pinhole: the exact FP64 coordinate rounded to FP32.  Spherical:
        // the coarse FP32 atan2 is within 6.1e-4 rad of each angle (6.09e-4 measured against the FP64
        // atan2 over 4e6 directions), scaled by |fx| or |fy| pixels per radian, plus the FP32 rounding of
        // fx a + cx (a few ulps of |cx| + |fx| pi).  The azimuth wraps at a = +-pi, i.e. at u' = cx -+ |fx| pi,
        // where the estimate may be a whole turn off; a wrap at least half a pixel outside the cells
        // [1, W - 3] leaves every point that can be valid within reach.
        d.early = 1;
        if (S.model == PBA_SPHERICAL) {
            const double pi = 3.14159265358979323846, afx = std::fabs(S.fx), afy = std::fabs(S.fy);
            const double eu = afx * 6.1e-4 + 4.0 * std::ldexp(std::fabs(S.cx) + afx * pi, -24) + 1e-6;
            const double ev = afy * 6.1e-4 + 4.0 * std::ldexp(std::fabs(S.cy) + afy * pi, -24) + 1e-6;
            auto off_cells = [&](double w) { return w <= 0.5 || w >= S.width - 1.5; };
            d.early = eu < 0.49 && ev < 0.49 && off_cells(S.cx - afx * pi) && off_cells(S.cx + afx * pi);
        }
        // the division-free coarse elevation: every row the image can reach (v' in (-1, H)) is below 45
        // degrees, so a point at 45 degrees or more is outside
        d.el45 = 0;
        if (S.model == PBA_SPHERICAL) {
            const double e0 = std::fabs((-1.0 - S.cy) / S.fy), e1 = std::fabs((S.height - S.cy) / S.fy);
            d.el45 = std::max(e0, e1) < 0.76;   // 43.5 degrees
        }
        for (int k = 0; k < 9; ++k) d.Ro[k] = S.offset[k];
        for (int k = 0; k < 3; ++k) d.to[k] = S.offset[9 + k];
        d.lut_col = (int64_t)l32.size();
        for (int u = 0; u < S.width; ++u) {
            double x, y;
            if (S.model == PBA_SPHERICAL) { const double az = (u - S.cx) / S.fx; x = std::cos(az); y = std::sin(az); }
            else { x = (u - S.cx) / S.fx; y = 0.0; }
            l32.push_back(make_float2((float)x, (float)y));
            l64.push_back(make_double2(x, y));
        }
        d.lut_row = (int64_t)l32.size();
        for (int v = 0; v < S.height; ++v) {
            double x, y;
            if (S.model == PBA_SPHERICAL) { const double el = (v - S.cy) / S.fy; x = std::cos(el); y = std::sin(el); }
            else { x = (v - S.cy) / S.fy; y = 0.0; }
            l32.push_back(make_float2((float)x, (float)y));
            l64.push_back(make_double2(x, y));
        }
    }
    pba_status s;
    if ((s = upload(c, is.sensors_d, sd.data(), sd.size() * sizeof(SensorDev)))) return s;
    if ((s = upload(c, is.lut32, l32.data(), l32.size() * sizeof(float2)))) return s;
    if ((s = upload(c, is.lut64, l64.data(), l64.size() * sizeof(double2)))) return s;
    is.sensors_dev_h = sd;
    return PBA_OK;
}

// Keyframe layout of one level: keyframes back to back in each plane.
pba_status image_layout(pba_ctx *c, ImageSet &is, const std::vector<int32_t> &sensor_of)
{
    is.kfs_h.assign(sensor_of.size(), KfDev{});
    int64_t off = 0;
    for (size_t k = 0; k < sensor_of.size(); ++k) {
        KfDev &f = is.kfs_h[k];
        f.sensor = sensor_of[k];
        f.H = is.sensors[f.sensor].height;
        f.W = is.sensors[f.sensor].width;
        f.pose = pose_var(c, (int)k);
        f.off = off;
        off += (int64_t)f.H * f.W;
    }
    is.texels = off;
    pba_status s;
    if ((s = upload(c, is.kfs_d, is.kfs_h.data(), is.kfs_h.size() * sizeof(KfDev)))) return s;
    if ((s = ensure(c, is.dep, off * sizeof(float)))) return s;
    if ((s = ensure(c, is.gate, off * sizeof(float2)))) return s;
    if (c->cfg.channels == 5) return ensure(c, is.att4, off * att_bytes(c));
    return ensure(c, is.att1, off * att_bytes(c));
}

// The depth-interval plane of every spherical keyframe of a level (only spherical targets read it), from
// its depth plane (enqueued on the context stream; rebuilt whenever the depth plane is written).
void build_gate(pba_ctx *c, ImageSet &is)
{
    for (const KfDev &f : is.kfs_h)
        if (is.sensors_dev_h[f.sensor].model == MODEL_SPHERICAL)
            launch_gate_plane(P_<float>(is.dep) + f.off, P_<float2>(is.gate) + f.off, f.H, f.W,
                              is.sensors_dev_h[f.sensor].taud, c->stream);
}

// Tiles (64 x 64) of the Cholesky factor of the 6 NP x 6 NP system that can be nonzero: those
// holding part of a pose variable's own 6 x 6 block or of a pair's coupling block, and those the
// factorisation fills (tile (i, j), i >= j, once tiles (i, k) and (j, k) are nonzero for some
// k < j).  The damped, gauge-fixed matrix has no nonzero outside this pattern, so the panel,
// trailing update and triangular solves may skip every other tile.
//
// In the natural order the factorisation is a chain of one dependent step per block column.  A
// nested-dissection order of the pose graph (blocks padded to 64 rows) lets the columns of one
// elimination-tree level factor in one launch; it is taken (solve_order auto) when it at least
// halves the chain without more than doubling the system's order, or always (solve_order nd).
void drop_graph(pba_ctx *c);

constexpr int kNdLeaf = 20;   // pose variables per dissection leaf (120 rows: two tiles)

// (A captured iteration holds the list pointers and launch counts, so it is dropped.)
pba_status build_chol_plan(pba_ctx *c, const std::vector<int32_t> &src, const std::vector<int32_t> &tgt)
{
    drop_graph(c);
    const int np = c->NP, n0 = n_sys(c);
    std::vector<std::pair<int, int>> edges(src.size());
    for (size_t p = 0; p < src.size(); ++p) edges[p] = {pose_var(c, src[p]), pose_var(c, tgt[p])};
    std::vector<int> pos(np);
    for (int v = 0; v < np; ++v) pos[v] = 6 * v;
    TilePattern tp = tile_pattern(n0, pos, edges);
    bool nd = false;
    if (c->cfg.solve_order != PBA_ORDER_NATURAL && np > 1) {
        int n_pad = 0;
        std::vector<int> pnd = nd_positions(np, nd_blocks(np, edges, kNdLeaf), n_pad);
        TilePattern t2 = tile_pattern(n_pad, pnd, edges);
        if (c->cfg.solve_order == PBA_ORDER_ND || (2 * t2.nlev <= tp.nt && n_pad <= 2 * n0 + 64)) {
            tp = std::move(t2);
            pos = std::move(pnd);
            nd = true;
        }
    }
    const int nt = tp.nt, n = tp.n;
    std::vector<int32_t> rows, cols;
    CholPlan &pl = c->chol;
    pl.rbeg.assign(nt, 0);
    pl.rcnt.assign(nt, 0);
    pl.cbeg.assign(nt, 0);
    pl.ccnt.assign(nt, 0);
    for (int k = 0; k < nt; ++k) {
        pl.rbeg[k] = (int)rows.size();
        rows.insert(rows.end(), tp.rows[k].begin(), tp.rows[k].end());
        pl.rcnt[k] = (int)tp.rows[k].size();
        pl.cbeg[k] = (int)cols.size();
        cols.insert(cols.end(), tp.cols[k].begin(), tp.cols[k].end());
        pl.ccnt[k] = (int)tp.cols[k].size();
    }
    const std::vector<int32_t> crows = rows, ccols = cols;
    rows.push_back(0);   // keep the device arrays non-empty
    cols.push_back(0);
    pba_status s;
    if ((s = upload(c, c->chol_rows, rows.data(), rows.size() * 4))) return s;
    if ((s = upload(c, c->chol_cols, cols.data(), cols.size() * 4))) return s;
    std::vector<int32_t> meta;
    for (const std::vector<int> *v : {&pl.rbeg, &pl.rcnt, &pl.cbeg, &pl.ccnt}) meta.insert(meta.end(), v->begin(), v->end());
    // the first kCholPre tile rows of each block column, then the first tile columns of each block
    // row, -1 padded
    for (int k = 0; k < nt; ++k)
        for (int e = 0; e < kCholPre; ++e) meta.push_back(e < pl.rcnt[k] ? crows[pl.rbeg[k] + e] : -1);
    for (int k = 0; k < nt; ++k)
        for (int e = 0; e < kCholPre; ++e) meta.push_back(e < pl.ccnt[k] ? ccols[pl.cbeg[k] + e] : -1);
    if ((s = upload(c, c->chol_meta, meta.data(), meta.size() * 4))) return s;
    pl.rows = P_<int32_t>(c->chol_rows);
    pl.cols = P_<int32_t>(c->chol_cols);
    pl.meta = P_<int32_t>(c->chol_meta);
    pl.np = np;
    pl.n = n;
    pl.nd = nd;
    pl.lbeg.clear();
    pl.lcnt.clear();
    pl.tbeg.clear();
    pl.tcnt.clear();
    pl.ndt = 0;
    if (nd) {
        const NdArrays a = nd_arrays(tp, pos);
        pl.lbeg = a.lbeg;
        pl.lcnt = a.lcnt;
        pl.tbeg = a.tbeg;
        pl.tcnt = a.tcnt;
        std::vector<int32_t> perm = a.perm, dtiles = a.dtiles, lcols = a.lcols, tasks = a.tasks, contrib = a.contrib;
        pl.ndt = (int)dtiles.size() / 2;
        contrib.push_back(0);
        tasks.insert(tasks.end(), {0, 0, 0, 0});
        if ((s = upload(c, c->nd_perm, perm.data(), perm.size() * 4))) return s;
        if ((s = upload(c, c->nd_off, pos.data(), pos.size() * 4))) return s;
        if ((s = upload(c, c->nd_dtiles, dtiles.data(), dtiles.size() * 4))) return s;
        if ((s = upload(c, c->nd_lcols, lcols.data(), lcols.size() * 4))) return s;
        if ((s = upload(c, c->nd_tasks, tasks.data(), tasks.size() * 4))) return s;
        if ((s = upload(c, c->nd_contrib, contrib.data(), contrib.size() * 4))) return s;
        if ((s = ensure(c, c->dx_nat, (size_t)n0 * 8))) return s;
        pl.perm = P_<int32_t>(c->nd_perm);
        pl.pose_off = P_<int32_t>(c->nd_off);
        pl.dtiles = P_<int32_t>(c->nd_dtiles);
        pl.lcols = P_<int32_t>(c->nd_lcols);
        pl.tasks = P_<int32_t>(c->nd_tasks);
        pl.contrib = P_<int32_t>(c->nd_contrib);
    }
    // the factorisation's buffers at the factored order: working matrix, the factor's panels and
    // their transposes; the inverted diagonal blocks (64 x 64 each, zero-padded) then their
    // transposes; the step
    const size_t nz = (size_t)n;
    if ((s = ensure(c, c->A, 3 * nz * nz * 8))) return s;
    if ((s = ensure(c, c->Winv, 2 * (size_t)nt * 64 * 64 * 8))) return s;
    if ((s = ensure(c, c->dx, nz * 8))) return s;
    return PBA_OK;
}

// The plan is dropped whenever the keyframes, the pose variables or the pairs change; rebuilt here
// from the pairs as set (none before any are set).
pba_status ensure_chol_plan(pba_ctx *c)
{
    if (c->chol.rows && c->chol.np == c->NP) return PBA_OK;
    const std::vector<int32_t> none;
    return c->P > 0 ? build_chol_plan(c, c->src_h, c->tgt_h) : build_chol_plan(c, none, none);
}

pba_status build_plan(pba_ctx *c, const std::vector<int32_t> &src, const std::vector<int32_t> &tgt)
{
    const int P = (int)src.size();
    // work items: (pair, first source pixel); grouped by (source model, target model),
    // ordered by target keyframe so items sharing a target image run close together
    std::vector<int> order(P);
    for (int p = 0; p < P; ++p) order[p] = p;
    auto model_of = [&](int kf) { return c->sensors[c->L().kfs_h[kf].sensor].model; };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        const int ka = model_of(src[a]) * 2 + model_of(tgt[a]), kb = model_of(src[b]) * 2 + model_of(tgt[b]);
        if (ka != kb) return ka < kb;
        return tgt[a] < tgt[b];
    });
    // items: (pair, first pixel); ordered by (model group, target keyframe, pixel band, pair) so
    // that concurrently processed items read the same rows of the same target images
    struct It { int key, tgt, band, pair, px; };
    std::vector<It> items;
    for (int oi = 0; oi < P; ++oi) {
        const int p = order[oi];
        const int key = model_of(src[p]) * 2 + model_of(tgt[p]);
        const int npx = c->L().kfs_h[src[p]].H * c->L().kfs_h[src[p]].W;
        for (int px = 0, band = 0; px < npx; px += c->items_px, ++band) items.push_back({key, tgt[p], band, p, px});
    }
    std::stable_sort(items.begin(), items.end(), [](const It &a, const It &b) {
        if (a.key != b.key) return a.key < b.key;
        if (a.tgt != b.tgt) return a.tgt < b.tgt;
        if (a.band != b.band) return a.band < b.band;
        return a.pair < b.pair;
    });
    std::vector<int32_t> ipair(items.size()), ipx(items.size());
    c->groups.clear();
    std::vector<std::vector<int32_t>> per_pair(P);
    for (size_t i = 0; i < items.size(); ++i) {
        const It &t = items[i];
        ipair[i] = t.pair;
        ipx[i] = t.px;
        per_pair[t.pair].push_back((int32_t)i);
        if (c->groups.empty() || c->groups.back().sm * 2 + c->groups.back().tm != t.key)
            c->groups.push_back({t.key >> 1, t.key & 1, (int)i, 0});
        c->groups.back().count = (int)i + 1 - c->groups.back().base;
    }
    // each pair's items in pixel order (the per-pair reduction sums them in this order)
    std::vector<int32_t> pitems;
    c->pair_item_begin.assign(P, 0);
    c->pair_item_count.assign(P, 0);
    for (int p = 0; p < P; ++p) {
        std::sort(per_pair[p].begin(), per_pair[p].end(), [&](int32_t a, int32_t b) { return ipx[a] < ipx[b]; });
        c->pair_item_begin[p] = (int32_t)pitems.size();
        c->pair_item_count[p] = (int32_t)per_pair[p].size();
        pitems.insert(pitems.end(), per_pair[p].begin(), per_pair[p].end());
    }
    c->n_items = (int)ipair.size();
    pba_status s;
    if ((s = upload(c, c->item_pair, ipair.data(), ipair.size() * 4))) return s;
    if ((s = upload(c, c->item_px0, ipx.data(), ipx.size() * 4))) return s;
    if ((s = upload(c, c->pitems, pitems.data(), pitems.size() * 4))) return s;
    if ((s = upload(c, c->ibeg, c->pair_item_begin.data(), P * 4))) return s;
    if ((s = upload(c, c->icnt, c->pair_item_count.data(), P * 4))) return s;
    if ((s = ensure(c, c->partials, (size_t)std::max(1, c->n_items) * kAcc * sizeof(double)))) return s;
    if ((s = ensure(c, c->pair_out, (size_t)std::max(1, P) * kPairOut * 8))) return s;
    if ((s = ensure(c, c->pair_dev, (size_t)std::max(1, P) * sizeof(PairDev)))) return s;

    // assembly plan: contributions of each nonzero 6x6 block, in pair order
    std::map<std::pair<int, int>, std::vector<int32_t>> blocks;
    // keyed by pose variable: a pair inside one rig frame adds all four blocks to its diagonal
    std::vector<std::vector<int32_t>> bk(c->NP);
    for (int p = 0; p < P; ++p) {
        const int a = pose_var(c, src[p]), t = pose_var(c, tgt[p]);
        blocks[{a, a}].push_back(4 * p + 0);
        blocks[{a, t}].push_back(4 * p + 1);
        blocks[{t, a}].push_back(4 * p + 2);
        blocks[{t, t}].push_back(4 * p + 3);
        bk[a].push_back(2 * p + 0);
        bk[t].push_back(2 * p + 1);
    }
    std::vector<int2> rc;
    std::vector<int32_t> ptr(1, 0), ent;
    for (auto &kv : blocks) {
        std::vector<int32_t> v = kv.second;
        std::stable_sort(v.begin(), v.end());
        rc.push_back(make_int2(kv.first.first, kv.first.second));
        ent.insert(ent.end(), v.begin(), v.end());
        ptr.push_back((int32_t)ent.size());
    }
    c->nblk = (int)rc.size();
    std::vector<int32_t> bptr(1, 0), bent;
    for (int k = 0; k < c->NP; ++k) {
        bent.insert(bent.end(), bk[k].begin(), bk[k].end());
        bptr.push_back((int32_t)bent.size());
    }
    if ((s = upload(c, c->blk_rc, rc.data(), rc.size() * sizeof(int2)))) return s;
    if ((s = upload(c, c->blk_ptr, ptr.data(), ptr.size() * 4))) return s;
    if ((s = upload(c, c->blk_ent, ent.data(), ent.size() * 4))) return s;
    if ((s = upload(c, c->bk_ptr, bptr.data(), bptr.size() * 4))) return s;
    if ((s = upload(c, c->bk_ent, bent.data(), bent.size() * 4))) return s;
    if ((s = ensure(c, c->counters, 64 * 4 * kCtrStride))) return s;
    if (c->cfg.occlusion_zbuffer) {   // one z-buffer per pair, sized for its target at this level
        std::vector<int64_t> zo(std::max(P, 1), 0);
        int64_t tot = 0;
        for (int p = 0; p < P; ++p) {
            zo[p] = tot;
            tot += (int64_t)c->L().kfs_h[tgt[p]].H * c->L().kfs_h[tgt[p]].W;
        }
        if ((s = upload(c, c->zoff, zo.data(), zo.size() * 8))) return s;
        if ((s = ensure(c, c->zbuf, (size_t)(tot + 2) * 4))) return s;   // whole doubles for the fill
        c->zcells = tot;
    }
    return build_chol_plan(c, src, tgt);
}

EvalArgs make_args(pba_ctx *c)
{
    EvalArgs a{};
    a.sensors = P_<SensorDev>(c->L().sensors_d);
    a.kfs = P_<KfDev>(c->L().kfs_d);
    a.pairs = P_<PairDev>(c->pair_dev);
    a.dep = P_<float>(c->L().dep);
    a.att4 = P_<float4>(c->L().att4);
    a.att1 = P_<float>(c->L().att1);
    a.att4h = P_<ushort4>(c->L().att4);
    a.att1h = P_<uint16_t>(c->L().att1);
    a.bf16 = c->cfg.storage_bf16;
    a.lut32 = P_<float2>(c->L().lut32);
    a.lut64 = P_<double2>(c->L().lut64);
    a.lut64_bytes = (int32_t)c->L().lut64.bytes;
    a.gate = P_<float2>(c->L().gate);
    a.item_pair = P_<int32_t>(c->item_pair);
    a.item_px0 = P_<int32_t>(c->item_px0);
    a.items_px = c->items_px;
    a.partials = c->partials.p;
    a.omega_g = c->cfg.omega_intensity;
    a.omega_d = c->cfg.omega_depth;
    a.omega_n = c->cfg.omega_normal;
    a.huber = c->cfg.huber_delta;
    if (c->cfg.occlusion_zbuffer) {
        a.zbuf = P_<uint32_t>(c->zbuf);
        a.zoff = P_<int64_t>(c->zoff);
    }
    return a;
}

// z-buffer occlusion variant: every pair's z-buffer at the poses the last pair setup used (+inf, then
// the nearest predicted depth per target cell by a projection-only pass of the evaluation kernel),
// then the pair setup again, which clears the queue counters for the evaluation proper.
// Working memory of one evaluation: queue counters (kXcd per model group), per-item partial sums
// and per-pair records.  The context's own buffers, or a caller-independent array (the
// allocation-free entry point).
struct WorkBufs {
    uint32_t *counters;
    void *partials;
    double *pair_out;
};

WorkBufs ctx_work(pba_ctx *c) { return WorkBufs{P_<uint32_t>(c->counters), c->partials.p, P_<double>(c->pair_out)}; }

void zbuffer_pass(pba_ctx *c, const double *poses, hipStream_t st, const WorkBufs &w)
{
    if (!c->cfg.occlusion_zbuffer || c->P == 0) return;
    const uint64_t inf2 = 0x7F8000007F800000ull;   // two FP32 +inf (a finite double)
    double fill;
    std::memcpy(&fill, &inf2, 8);
    launch_fill(P_<double>(c->zbuf), (c->zcells + 1) / 2, fill, st);
    EvalArgs a = make_args(c);
    a.partials = w.partials;
    a.zpass = 1;
    const int ngrp = (int)c->groups.size();
    for (int g = 0; g < ngrp; ++g) {
        const auto &G = c->groups[g];
        a.counter = w.counters + g * kXcd * kCtrStride;
        launch_eval(a, c->cfg.precision, c->cfg.channels, c->cfg.grad_mode, G.sm, G.tm, false, G.base, G.count,
                    std::max(1, std::min(G.count, c->grid)), st);
    }
    launch_pair_setup(poses, P_<int2>(c->pairs_d), c->P, P_<SensorDev>(c->L().sensors_d), P_<KfDev>(c->L().kfs_d),
                      P_<PairDev>(c->pair_dev), w.counters, ngrp * kXcd, st);
}

// Evaluate at `poses` into (H, b, totals).  Launch order on the context stream:
// pair setup (also clears the queue counters) -> persistent evaluation per model group
// -> ordered per-pair reduction/expansion -> assembly.  `timed` brackets the evaluation launches
// with the context's HIP events; `stamped` with wall-clock stamps into the LM log row (for
// launches inside a captured iteration, where the events would only keep the last replay).
pba_status run_eval(pba_ctx *c, const double *poses, double *H, double *b, double *totals, bool timed,
                    hipStream_t st, bool stamped = false, const WorkBufs *work = nullptr)
{
    const WorkBufs w = work ? *work : ctx_work(c);
    const int ngrp = (int)c->groups.size();
    launch_pair_setup(poses, P_<int2>(c->pairs_d), c->P, P_<SensorDev>(c->L().sensors_d), P_<KfDev>(c->L().kfs_d),
                      P_<PairDev>(c->pair_dev), w.counters, ngrp * kXcd, st);
    zbuffer_pass(c, poses, st, w);
    EvalArgs a = make_args(c);
    a.partials = w.partials;
    if (timed) HIP_OK(hipEventRecord(c->ev0, st));
    if (stamped) launch_stamp(P_<LmState>(c->lm), P_<double>(c->logbuf), c->log_cap, 0, st);
    for (int g = 0; g < ngrp; ++g) {
        const auto &G = c->groups[g];
        a.counter = w.counters + g * kXcd * kCtrStride;
        const int grid = std::max(1, std::min(G.count, c->grid));
        launch_eval(a, c->cfg.precision, c->cfg.channels, c->cfg.grad_mode, G.sm, G.tm, false, G.base, G.count, grid,
                    st);
    }
    if (timed) HIP_OK(hipEventRecord(c->ev1, st));
    if (stamped) launch_stamp(P_<LmState>(c->lm), P_<double>(c->logbuf), c->log_cap, 1, st);
    HIP_OK(hipGetLastError());
    launch_reduce_pairs(w.partials, c->cfg.precision, P_<int32_t>(c->pitems), P_<int32_t>(c->ibeg),
                        P_<int32_t>(c->icnt), P_<PairDev>(c->pair_dev), w.pair_out, c->P, st);
    launch_assemble(w.pair_out, c->P, P_<int2>(c->blk_rc), P_<int32_t>(c->blk_ptr),
                    P_<int32_t>(c->blk_ent), c->nblk, P_<int32_t>(c->bk_ptr), P_<int32_t>(c->bk_ent), c->NP, H, b,
                    totals, st);
    HIP_OK(hipGetLastError());
    return PBA_OK;
}

void drop_graph(pba_ctx *c)
{
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->gexec = nullptr;
    c->graph = nullptr;
    c->graph_valid = false;
}

// Damped, gauge-fixed solve of the current system into dx (the plan's order and layout): lambda
// from lm, or lam_override when >= 0.
void enqueue_solve(pba_ctx *c, const LmState *lm, double lam_override, hipStream_t st)
{
    const CholPlan &pl = c->chol;
    const int n = pl.n;
    double *A = P_<double>(c->A), *Lf = A + (size_t)n * n, *LTf = Lf + (size_t)n * n;
    if (pl.nd)
        launch_damp_copy_perm(P_<double>(c->H), P_<double>(c->b), A, P_<double>(c->dx), n_sys(c), c->cfg.anchor, lm,
                              lam_override, pl, P_<int32_t>(c->fail), st);
    else
        launch_damp_copy(P_<double>(c->H), P_<double>(c->b), A, P_<double>(c->dx), n, c->cfg.anchor, lm,
                         lam_override, st);
    launch_cholesky(A, Lf, LTf, n, P_<double>(c->Winv), pl, P_<int32_t>(c->fail), st, P_<double>(c->dx));
    launch_chol_solve(Lf, LTf, P_<double>(c->Winv), P_<double>(c->dx), n, pl, P_<int32_t>(c->fail), st);
}

// Enqueue one LM / GN iteration on `st`: damped solve at the current poses, candidate poses,
// evaluation at the candidate, device-side accept/reject.  Identical launches every iteration.
pba_status enqueue_iteration(pba_ctx *c, hipStream_t st)
{
    const int n = n_sys(c);
    double *totals = P_<double>(c->totals);   // [0..3] current, [4..7] candidate
    launch_stamp(P_<LmState>(c->lm), P_<double>(c->logbuf), c->log_cap, 2, st);
    enqueue_solve(c, P_<LmState>(c->lm), -1.0, st);
    launch_boxplus(P_<double>(c->poses), P_<double>(c->dx), c->chol.nd ? c->chol.pose_off : nullptr,
                   P_<double>(c->poses_cand), c->NP, P_<int32_t>(c->fail), P_<LmState>(c->lm), st);
    pba_status s = run_eval(c, P_<double>(c->poses_cand), P_<double>(c->H_cand), P_<double>(c->b_cand), totals + 4,
                            false, st, true);
    if (s) return s;
    launch_lm_decide(P_<LmState>(c->lm), totals + 4, (int64_t)n * n, P_<double>(c->H), P_<double>(c->H_cand),
                     P_<double>(c->b), P_<double>(c->b_cand), P_<double>(c->poses), P_<double>(c->poses_cand), c->NP,
                     totals, P_<double>(c->logbuf), c->log_cap, st);
    HIP_OK(hipGetLastError());
    return PBA_OK;
}

pba_status accumulate_eval_time(pba_ctx *c)
{
    HIP_OK(hipEventSynchronize(c->ev1));
    float ms = 0.f;
    HIP_OK(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    c->eval_ms += ms;
    c->eval_launches += 1;
    return PBA_OK;
}

void *att_plane(pba_ctx *c, ImageSet &is) { return c->cfg.channels == 5 ? is.att4.p : is.att1.p; }

size_t att_bytes(const pba_ctx *c)
{
    if (c->cfg.channels == 5) return c->cfg.storage_bf16 ? sizeof(ushort4) : sizeof(float4);
    return c->cfg.storage_bf16 ? sizeof(uint16_t) : sizeof(float);
}

pba_status check_ready(pba_ctx *c)
{
    if (c->N == 0) return fail(c, PBA_ESTATE, "no keyframes loaded");
    if (!c->poses_set) return fail(c, PBA_ESTATE, "poses not set");
    if (c->P == 0) return fail(c, PBA_ESTATE, "pairs not set");
    return PBA_OK;
}

pba_status ensure_system(pba_ctx *c)
{
    const size_t n = (size_t)n_sys(c);
    pba_status s;
    if ((s = ensure(c, c->H, n * n * 8))) return s;
    if ((s = ensure(c, c->b, n * 8))) return s;
    if ((s = ensure(c, c->totals, 8 * 8))) return s;
    if ((s = ensure(c, c->A, 3 * n * n * 8))) return s;   // working matrix, the factor's panels, their transposes
    if ((s = ensure(c, c->H_cand, n * n * 8))) return s;
    if ((s = ensure(c, c->b_cand, n * 8))) return s;
    // inverted diagonal blocks, 64 x 64 each, zero-padded, then their transposes
    if ((s = ensure(c, c->Winv, 2 * ((n + 63) / 64) * 64 * 64 * 8))) return s;
    if ((s = ensure(c, c->dx, n * 8))) return s;
    if ((s = ensure(c, c->lm, sizeof(LmState)))) return s;
    if ((s = ensure(c, c->fail, 16))) return s;
    return PBA_OK;
}

}  // namespace

extern "C" {

void pba_config_default(pba_config *cfg)
{
    if (!cfg) return;
    std::memset(cfg, 0, sizeof *cfg);
    cfg->device = 0;
    cfg->precision = PBA_F32;
    cfg->channels = 5;
    cfg->grad_mode = 0;
    cfg->anchor = 0;
    cfg->use_graph = 1;
    cfg->stream = nullptr;
    cfg->omega_intensity = 1.0;
    cfg->omega_depth = 1.0;
    cfg->omega_normal = 1.0;
    cfg->huber_delta = 0.1;
    cfg->occlusion_tau_pinhole = 0.5;
    cfg->occlusion_tau_spherical = 1.0;
}

const char *pba_status_string(pba_status s)
{
    switch (s) {
    case PBA_OK: return "ok";
    case PBA_EINVAL: return "invalid argument";
    case PBA_ENOMEM: return "out of device memory";
    case PBA_EDEVICE: return "HIP device error";
    case PBA_ESTATE: return "call out of order";
    case PBA_ENOTPD: return "system not positive definite";
    case PBA_ENOVALID: return "no valid correspondence";
    default: return "unknown status";
    }
}

const char *pba_last_error(const pba_ctx *c) { return c ? c->err.c_str() : "null context"; }

pba_status pba_create(const pba_config *cfg, pba_ctx **out)
{
    if (!cfg || !out) return PBA_EINVAL;
    *out = nullptr;
    if (cfg->precision != PBA_F32 && cfg->precision != PBA_F64) return PBA_EINVAL;
    if (cfg->channels != 2 && cfg->channels != 5) return PBA_EINVAL;
    if (cfg->grad_mode != 0 && cfg->grad_mode != 1) return PBA_EINVAL;
    if (cfg->anchor < 0) return PBA_EINVAL;
    const double w[6] = {cfg->omega_intensity, cfg->omega_depth, cfg->omega_normal, cfg->huber_delta,
                         cfg->occlusion_tau_pinhole, cfg->occlusion_tau_spherical};
    for (double x : w)
        if (!std::isfinite(x)) return PBA_EINVAL;
    if (cfg->omega_intensity < 0 || cfg->omega_depth < 0 || cfg->omega_normal < 0) return PBA_EINVAL;
    if (!(cfg->occlusion_tau_pinhole > 0) || !(cfg->occlusion_tau_spherical > 0)) return PBA_EINVAL;
    if (cfg->occlusion_zbuffer != 0 && cfg->occlusion_zbuffer != 1) return PBA_EINVAL;
    // BF16 storage: FP32 evaluation path only, without the z-buffer variant
    if (cfg->storage_bf16 != 0 && cfg->storage_bf16 != 1) return PBA_EINVAL;
    if (cfg->storage_bf16 && (cfg->precision != PBA_F32 || cfg->occlusion_zbuffer)) return PBA_EINVAL;
    if (cfg->solve_order < PBA_ORDER_AUTO || cfg->solve_order > PBA_ORDER_ND) return PBA_EINVAL;
    if ((cfg->dev_alloc == nullptr) != (cfg->dev_free == nullptr)) return PBA_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || cfg->device < 0 || cfg->device >= ndev) return PBA_EDEVICE;
    if (hipSetDevice(cfg->device) != hipSuccess) return PBA_EDEVICE;
    if (cfg->device >= kMaxDevices) return PBA_EDEVICE;
    {
        // the device address of this GPU's copy of the scratch array (pba_evaluate_noalloc)
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch_ptr[cfg->device]) {
            void *p = nullptr;
            if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return PBA_EDEVICE;
            g_scratch_ptr[cfg->device] = p;
        }
    }
    pba_ctx *c = new (std::nothrow) pba_ctx;
    if (!c) return PBA_ENOMEM;
    c->cfg = *cfg;
    c->stream = static_cast<hipStream_t>(cfg->stream);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, cfg->device) == hipSuccess && prop.multiProcessorCount > 0)
        c->num_cu = prop.multiProcessorCount;
    c->grid = c->num_cu * 4;
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, cfg->device) == hipSuccess && khz > 0)
        c->wall_khz = khz;
    if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess) {
        delete c;
        return PBA_EDEVICE;
    }
    *out = c;
    return PBA_OK;
}

pba_status pba_destroy(pba_ctx *c)
{
    if (!c) return PBA_EINVAL;
    (void)hipSetDevice(c->cfg.device);
    (void)hipStreamSynchronize(c->stream);
    for (ImageSet &is : c->lv) release_images(is);
    DevBuf *bufs[] = {&c->poses, &c->poses_cand, &c->pairs_d, &c->pair_dev, &c->item_pair, &c->item_px0, &c->pitems, &c->ibeg, &c->icnt,
                      &c->counters, &c->partials, &c->pair_out, &c->blk_rc, &c->blk_ptr, &c->blk_ent, &c->bk_ptr,
                      &c->bk_ent, &c->H, &c->b, &c->H_cand, &c->b_cand, &c->totals, &c->A, &c->Winv, &c->dx, &c->lm,
                      &c->fail, &c->logbuf, &c->dbg_status, &c->dbg_uv, &c->dbg_cell, &c->dbg_res,
                      &c->loss_delta, &c->loss_poses, &c->g_int, &c->g_dep, &c->g_nrm, &c->g_pose,
                      &c->chol_rows, &c->chol_cols, &c->chol_meta, &c->zbuf, &c->zoff, &c->nd_perm,
                      &c->nd_off, &c->nd_dtiles, &c->nd_lcols, &c->nd_tasks, &c->nd_contrib, &c->dx_nat};
    drop_graph(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    for (DevBuf *b : bufs) release(*b);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    delete c;
    return PBA_OK;
}

pba_status pba_add_sensor(pba_ctx *c, const pba_sensor *s, int32_t *sensor_id)
{
    if (!c || !s) return fail(c, PBA_EINVAL, "null argument");
    if (c->N > 0) return fail(c, PBA_ESTATE, "sensors must be added before keyframes are loaded");
    if (s->model != PBA_PINHOLE && s->model != PBA_SPHERICAL) return fail(c, PBA_EINVAL, "unknown sensor model");
    // the kernels split a pixel index into (row, col) with a 32-bit reciprocal multiply, exact
    // while H * W^2 < 2^32, and address one keyframe plane (16 B per texel) with 32-bit byte
    // offsets, so H * W <= 2^26
    if (s->height < 4 || s->width < 4 || (uint64_t)s->height * s->width * s->width >= (1ull << 32) ||
        (uint64_t)s->height * s->width > (1ull << 26))
        return fail(c, PBA_EINVAL, "image size %d x %d out of range", s->height, s->width);
    const double v[6] = {s->fx, s->fy, s->cx, s->cy, s->min_depth, s->max_depth};
    for (double x : v)
        if (!std::isfinite(x)) return fail(c, PBA_EINVAL, "non-finite intrinsics");
    if (s->fx == 0.0 || s->fy == 0.0) return fail(c, PBA_EINVAL, "zero focal length / resolution");
    // the evaluation's coarse FP32 projection (within 6.1e-4 rad) must land within a pixel of the exact one
    if (s->model == PBA_SPHERICAL && std::max(std::fabs(s->fx), std::fabs(s->fy)) * 6.1e-4 >= 0.95)
        return fail(c, PBA_EINVAL, "spherical resolution %.0f px/rad above 1550", std::max(std::fabs(s->fx), std::fabs(s->fy)));
    if (!(s->min_depth > 0.0 && s->max_depth > s->min_depth)) return fail(c, PBA_EINVAL, "bad depth interval");
    if (!pose_ok(s->offset)) return fail(c, PBA_EINVAL, "sensor offset is not a rigid transform");
    c->sensors.push_back(*s);
    if (sensor_id) *sensor_id = (int32_t)c->sensors.size() - 1;
    return PBA_OK;
}

pba_status pba_load_keyframes(pba_ctx *c, int32_t n, const int32_t *sensor_id, const float *const *intensity,
                              const float *const *depth, const float *const *normals, int32_t on_device)
{
    if (!c) return PBA_EINVAL;
    if (n <= 0 || !sensor_id || !intensity || !depth) return fail(c, PBA_EINVAL, "bad keyframe arguments");
    if (c->sensors.empty()) return fail(c, PBA_ESTATE, "no sensor registered");
    if (c->cfg.channels == 5 && !normals) return fail(c, PBA_EINVAL, "5 channels need normals");
    HIP_OK(hipSetDevice(c->cfg.device));
    std::vector<int32_t> sensor_of(n);
    for (int k = 0; k < n; ++k) {
        const int sid = sensor_id[k];
        if (sid < 0 || sid >= (int)c->sensors.size()) return fail(c, PBA_EINVAL, "keyframe %d: bad sensor id", k);
        if (!intensity[k] || !depth[k] || (c->cfg.channels == 5 && !normals[k]))
            return fail(c, PBA_EINVAL, "keyframe %d: null image", k);
        sensor_of[k] = sid;
    }
    pba_status s;
    const int prev_level = c->level;
    const bool same_layout = c->N == n && (int)c->lv[0].kfs_h.size() == n &&
                             std::equal(sensor_of.begin(), sensor_of.end(), c->lv[0].kfs_h.begin(),
                                        [](int32_t a, const KfDev &f) { return a == f.sensor; });
    // a new load drops any pyramid: level 0 becomes the only and active level
    for (size_t l = 1; l < c->lv.size(); ++l) release_images(c->lv[l]);
    c->lv.resize(1);
    c->level = 0;
    ImageSet &is = c->lv[0];
    is.sensors = c->sensors;
    if ((s = sensor_tables(c, is))) return s;
    if (!same_layout) c->pose_of.clear();   // a new keyframe set starts with one pose per keyframe
    if ((s = image_layout(c, is, sensor_of))) return s;
    const std::vector<KfDev> &kfs = is.kfs_h;
    // stage each keyframe on the device (copy if host) and pack
    DevBuf stage;
    for (int k = 0; k < n; ++k) {
        const int npx = kfs[k].H * kfs[k].W;
        const pba_sensor &S = c->sensors[kfs[k].sensor];
        const float *dI = intensity[k], *dD = depth[k], *dN = c->cfg.channels == 5 ? normals[k] : nullptr;
        if (!on_device) {
            const size_t need = (size_t)npx * (c->cfg.channels == 5 ? 5 : 2) * 4;
            if ((s = ensure(c, stage, need))) { release(stage); return s; }
            float *base = P_<float>(stage);
            HIP_OK(hipMemcpyAsync(base, intensity[k], (size_t)npx * 4, hipMemcpyHostToDevice, c->stream));
            HIP_OK(hipMemcpyAsync(base + npx, depth[k], (size_t)npx * 4, hipMemcpyHostToDevice, c->stream));
            if (dN) HIP_OK(hipMemcpyAsync(base + 2 * (size_t)npx, normals[k], (size_t)npx * 12, hipMemcpyHostToDevice,
                                          c->stream));
            dI = base; dD = base + npx; dN = dN ? base + 2 * (size_t)npx : nullptr;
        }
        const int blocks = std::min((npx + 255) / 256, 4096);
        const bool five = c->cfg.channels == 5;
        hipLaunchKernelGGL(pack_kernel, dim3(blocks), dim3(256), 0, c->stream, dI, dD, five ? dN : nullptr,
                           P_<float>(c->L().dep) + kfs[k].off,
                           static_cast<char *>(att_plane(c, c->L())) + kfs[k].off * att_bytes(c), five ? 1 : 0,
                           c->cfg.storage_bf16, npx, S.min_depth, S.max_depth);
        if (!on_device) HIP_OK(hipStreamSynchronize(c->stream));   // stage is reused
    }
    build_gate(c, is);
    HIP_OK(hipGetLastError());
    HIP_OK(hipStreamSynchronize(c->stream));
    release(stage);
    drop_graph(c);
    c->system_valid = false;
    c->loss_ready = false;
    if (same_layout) {   // images replaced; poses and pairs kept (the plan follows level 0 again)
        if (prev_level != 0 && c->P > 0 && (s = build_plan(c, c->src_h, c->tgt_h))) return s;
        return PBA_OK;
    }
    c->N = n;
    c->NP = n;
    c->P = 0;
    c->chol.rows = nullptr;
    c->poses_set = false;
    if ((s = ensure(c, c->poses, (size_t)n * 12 * 8))) return s;
    if ((s = ensure(c, c->poses_cand, (size_t)n * 12 * 8))) return s;
    if (c->cfg.anchor >= n) return fail(c, PBA_EINVAL, "anchor %d >= number of keyframes %d", c->cfg.anchor, n);
    return PBA_OK;
}

pba_status pba_set_poses(pba_ctx *c, int32_t n, const double *poses, int32_t on_device)
{
    if (!c || !poses) return fail(c, PBA_EINVAL, "null argument");
    if (n != c->NP || n == 0) return fail(c, PBA_EINVAL, "expected %d poses, got %d", c->NP, n);
    std::vector<double> h((size_t)n * 12);
    HIP_OK(hipSetDevice(c->cfg.device));
    if (on_device) {
        HIP_OK(hipMemcpyAsync(h.data(), poses, h.size() * 8, hipMemcpyDeviceToHost, c->stream));
        HIP_OK(hipStreamSynchronize(c->stream));
    } else {
        std::memcpy(h.data(), poses, h.size() * 8);
    }
    for (int k = 0; k < n; ++k)
        if (!pose_ok(&h[12 * (size_t)k])) return fail(c, PBA_EINVAL, "pose %d is not finite/orthonormal", k);
    pba_status s = upload(c, c->poses, h.data(), h.size() * 8);
    if (s) return s;
    HIP_OK(hipStreamSynchronize(c->stream));
    c->poses_set = true;
    c->system_valid = false;
    c->lam_carry = -1.0;
    return PBA_OK;
}

pba_status pba_get_poses(pba_ctx *c, double *poses, int32_t on_device)
{
    if (!c || !poses) return fail(c, PBA_EINVAL, "null argument");
    if (!c->poses_set) return fail(c, PBA_ESTATE, "poses not set");
    HIP_OK(hipSetDevice(c->cfg.device));
    HIP_OK(hipMemcpyAsync(poses, c->poses.p, (size_t)c->NP * 96, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                          c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    return PBA_OK;
}

pba_status pba_set_pose_groups(pba_ctx *c, const int32_t *pose_of, int32_t n_poses)
{
    if (!c) return PBA_EINVAL;
    if (c->N == 0) return fail(c, PBA_ESTATE, "no keyframes loaded");
    std::vector<int32_t> g;
    int np = c->N;
    if (pose_of) {
        if (n_poses < 1 || n_poses > c->N) return fail(c, PBA_EINVAL, "n_poses %d not in 1..%d", n_poses, c->N);
        g.assign(pose_of, pose_of + c->N);
        std::vector<char> used(n_poses, 0);
        for (int k = 0; k < c->N; ++k) {
            if (g[k] < 0 || g[k] >= n_poses) return fail(c, PBA_EINVAL, "keyframe %d: pose variable %d out of range", k, g[k]);
            used[g[k]] = 1;
        }
        for (int v = 0; v < n_poses; ++v)
            if (!used[v]) return fail(c, PBA_EINVAL, "pose variable %d has no keyframe", v);
        np = n_poses;
    }
    if (c->cfg.anchor >= np) return fail(c, PBA_EINVAL, "anchor %d >= number of pose variables %d", c->cfg.anchor, np);
    HIP_OK(hipSetDevice(c->cfg.device));
    c->pose_of = g;
    c->NP = np;
    c->chol.rows = nullptr;
    pba_status s;
    for (ImageSet &is : c->lv) {
        for (int k = 0; k < c->N; ++k) is.kfs_h[k].pose = pose_var(c, k);
        if ((s = upload(c, is.kfs_d, is.kfs_h.data(), is.kfs_h.size() * sizeof(KfDev)))) return s;
    }
    drop_graph(c);
    c->poses_set = false;
    c->system_valid = false;
    c->loss_ready = false;
    c->lam_carry = -1.0;
    if (c->P > 0) {
        if ((s = build_plan(c, c->src_h, c->tgt_h))) return s;
        if ((s = ensure_system(c))) return s;
    }
    HIP_OK(hipStreamSynchronize(c->stream));
    return PBA_OK;
}

pba_status pba_set_pairs(pba_ctx *c, int32_t p, const int32_t *src, const int32_t *tgt)
{
    if (!c || (p > 0 && (!src || !tgt)) || p < 0) return fail(c, PBA_EINVAL, "bad pair arguments");
    if (c->N == 0) return fail(c, PBA_ESTATE, "no keyframes loaded");
    HIP_OK(hipSetDevice(c->cfg.device));
    std::vector<int32_t> s(src, src + p), t(tgt, tgt + p);
    for (int k = 0; k < p; ++k)
        if (s[k] < 0 || s[k] >= c->N || t[k] < 0 || t[k] >= c->N)
            return fail(c, PBA_EINVAL, "pair %d: keyframe id out of range", k);
    std::vector<int2> pr(p);
    for (int k = 0; k < p; ++k) pr[k] = make_int2(s[k], t[k]);
    drop_graph(c);
    pba_status st;
    if ((st = upload(c, c->pairs_d, pr.data(), pr.size() * sizeof(int2)))) return st;
    if ((st = build_plan(c, s, t))) return st;
    if ((st = ensure_system(c))) return st;
    HIP_OK(hipStreamSynchronize(c->stream));
    c->src_h = s;
    c->tgt_h = t;
    c->P = p;
    c->system_valid = false;
    c->lam_carry = -1.0;
    return PBA_OK;
}

pba_status pba_evaluate(pba_ctx *c, pba_eval_out *out)
{
    if (!c || !out) return fail(c, PBA_EINVAL, "null argument");
    pba_status s;
    if ((s = check_ready(c))) return s;
    HIP_OK(hipSetDevice(c->cfg.device));
    if ((s = run_eval(c, P_<double>(c->poses), P_<double>(c->H), P_<double>(c->b), P_<double>(c->totals), true, c->stream)))
        return s;
    const size_t n = (size_t)n_sys(c);
    const hipMemcpyKind k = out->on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (out->H) HIP_OK(hipMemcpyAsync(out->H, c->H.p, n * n * 8, k, c->stream));
    if (out->b) HIP_OK(hipMemcpyAsync(out->b, c->b.p, n * 8, k, c->stream));
    if (out->pair_out) HIP_OK(hipMemcpyAsync(out->pair_out, c->pair_out.p, (size_t)c->P * kPairOut * 8, k, c->stream));
    double tot[4];
    HIP_OK(hipMemcpyAsync(tot, c->totals.p, sizeof tot, hipMemcpyDeviceToHost, c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    if ((s = accumulate_eval_time(c))) return s;
    c->system_valid = true;
    out->F = tot[0];
    out->n_evaluated = (int64_t)tot[1];
    out->n_valid = (int64_t)tot[2];
    out->n_boundary_band = (int64_t)tot[3];
    return PBA_OK;
}

pba_status pba_evaluate_noalloc(pba_ctx *c, pba_eval_out *out)
{
    if (!c || !out) return fail(c, PBA_EINVAL, "null argument");
    pba_status s;
    if ((s = check_ready(c))) return s;
    HIP_OK(hipSetDevice(c->cfg.device));
    // carve the queue counters, per-item partials and per-pair records out of this device's array,
    // each part 256-byte aligned
    auto up = [](size_t n) { return (n + 255) & ~size_t(255); };
    const size_t n_cnt = up((size_t)std::max<size_t>(1, c->groups.size()) * kXcd * kCtrStride * 4);
    const size_t n_part = up((size_t)std::max(1, c->n_items) * kAcc * 8);
    const size_t n_pair = up((size_t)std::max(1, c->P) * kPairOut * 8);
    if (n_cnt + n_part + n_pair > kScratchBytes)
        return fail(c, PBA_EINVAL,
                    "pba_evaluate_noalloc: %d work items and %d pairs need %zu bytes of scratch, more than its %zu",
                    c->n_items, c->P, n_cnt + n_part + n_pair, kScratchBytes);
    unsigned char *base = static_cast<unsigned char *>(g_scratch_ptr[c->cfg.device]);
    if (!base) return fail(c, PBA_EDEVICE, "scratch array of device %d not resolved", c->cfg.device);
    const WorkBufs w{reinterpret_cast<uint32_t *>(base), base + n_cnt, reinterpret_cast<double *>(base + n_cnt + n_part)};
    if ((s = run_eval(c, P_<double>(c->poses), P_<double>(c->H), P_<double>(c->b), P_<double>(c->totals), false,
                      c->stream, false, &w)))
        return s;
    const size_t n = (size_t)n_sys(c);
    const hipMemcpyKind k = out->on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (out->H) HIP_OK(hipMemcpyAsync(out->H, c->H.p, n * n * 8, k, c->stream));
    if (out->b) HIP_OK(hipMemcpyAsync(out->b, c->b.p, n * 8, k, c->stream));
    if (out->pair_out) HIP_OK(hipMemcpyAsync(out->pair_out, w.pair_out, (size_t)c->P * kPairOut * 8, k, c->stream));
    double tot[4];
    HIP_OK(hipMemcpyAsync(tot, c->totals.p, sizeof tot, hipMemcpyDeviceToHost, c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    c->system_valid = true;
    out->F = tot[0];
    out->n_evaluated = (int64_t)tot[1];
    out->n_valid = (int64_t)tot[2];
    out->n_boundary_band = (int64_t)tot[3];
    return PBA_OK;
}

pba_status pba_solve_step(pba_ctx *c, double lambda, double *dx, int32_t on_device)
{
    if (!c) return PBA_EINVAL;
    if (!(lambda >= 0.0) || !std::isfinite(lambda)) return fail(c, PBA_EINVAL, "lambda must be finite and >= 0");
    pba_status s;
    if ((s = check_ready(c))) return s;
    HIP_OK(hipSetDevice(c->cfg.device));
    if ((s = ensure_chol_plan(c))) return s;
    const int n = n_sys(c);
    if (!c->system_valid) {
        if ((s = run_eval(c, P_<double>(c->poses), P_<double>(c->H), P_<double>(c->b), P_<double>(c->totals),
                          false, c->stream)))
            return s;
        c->system_valid = true;
    }
    enqueue_solve(c, P_<LmState>(c->lm), lambda, c->stream);
    // the step in pose order
    const double *step = P_<double>(c->dx);
    if (c->chol.nd && dx) {
        double *dst = on_device ? dx : P_<double>(c->dx_nat);
        launch_gather_step(dst, step, c->chol.pose_off, c->NP, c->stream);
        step = dst;
    }
    HIP_OK(hipGetLastError());
    int32_t f = 0;
    HIP_OK(hipMemcpyAsync(&f, c->fail.p, 4, hipMemcpyDeviceToHost, c->stream));
    if (dx && step != dx)
        HIP_OK(hipMemcpyAsync(dx, step, (size_t)n * 8, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                              c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    if (f) return fail(c, PBA_ENOTPD, "damped system is not positive definite (lambda = %g)", lambda);
    return PBA_OK;
}

pba_status pba_apply_step(pba_ctx *c, const double *dx, int32_t on_device)
{
    if (!c) return PBA_EINVAL;
    pba_status s;
    if ((s = check_ready(c))) return s;
    HIP_OK(hipSetDevice(c->cfg.device));
    const int n = n_sys(c);
    if (dx) {
        std::vector<double> h(n);
        if (on_device) {
            HIP_OK(hipMemcpyAsync(h.data(), dx, (size_t)n * 8, hipMemcpyDeviceToHost, c->stream));
            HIP_OK(hipStreamSynchronize(c->stream));
        } else {
            std::memcpy(h.data(), dx, (size_t)n * 8);
        }
        for (double v : h)
            if (!std::isfinite(v)) return fail(c, PBA_EINVAL, "non-finite step");
        if ((s = upload(c, c->dx, h.data(), (size_t)n * 8))) return s;
    }
    launch_boxplus(P_<double>(c->poses), P_<double>(c->dx), nullptr, P_<double>(c->poses_cand), c->NP, nullptr,
                   nullptr, c->stream);
    launch_copy(P_<double>(c->poses), P_<double>(c->poses_cand), (int64_t)c->NP * 12, c->stream);
    HIP_OK(hipGetLastError());
    HIP_OK(hipStreamSynchronize(c->stream));
    c->system_valid = false;
    c->lam_carry = -1.0;
    return PBA_OK;
}

pba_status pba_iterate(pba_ctx *c, int32_t n_iters, int32_t use_lm, double lambda0, pba_iter_log *log)
{
    if (!c) return PBA_EINVAL;
    if (n_iters < 0) return fail(c, PBA_EINVAL, "negative iteration count");
    if (use_lm && !(lambda0 >= 0.0 && std::isfinite(lambda0))) return fail(c, PBA_EINVAL, "bad lambda0");
    pba_status s;
    if ((s = check_ready(c))) return s;
    if (n_iters == 0) return PBA_OK;
    HIP_OK(hipSetDevice(c->cfg.device));
    if ((s = ensure_chol_plan(c))) return s;
    if (n_iters > c->log_cap) {
        const int cap = std::max(n_iters, 64);
        release(c->logbuf);
        if ((s = ensure(c, c->logbuf, (size_t)cap * kLogRow * 8))) return s;
        c->log_cap = cap;
        drop_graph(c);   // the graph refers to the log buffer
    }
    double *totals = P_<double>(c->totals);   // [0..3] current, [4..7] candidate
    // system at the current poses (reused if already evaluated there)
    if (!c->system_valid) {
        if ((s = run_eval(c, P_<double>(c->poses), P_<double>(c->H), P_<double>(c->b), totals, false, c->stream)))
            return s;
        c->system_valid = true;
    }
    double tot0[4];
    HIP_OK(hipMemcpyAsync(tot0, totals, sizeof tot0, hipMemcpyDeviceToHost, c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    LmState lm{};
    lm.lam = use_lm ? (lambda0 > 0.0 ? lambda0 : (c->lam_carry > 0.0 ? c->lam_carry : 1e-4)) : 0.0;
    lm.F_cur = tot0[0];
    lm.valid_cur = (int64_t)tot0[2];
    lm.use_lm = use_lm ? 1 : 0;
    HIP_OK(hipMemcpyAsync(c->lm.p, &lm, sizeof lm, hipMemcpyHostToDevice, c->stream));
    HIP_OK(hipEventRecord(c->ev0, c->stream));
    if (c->cfg.use_graph) {
        if (!c->graph_valid) {
            if (!c->cap_stream) HIP_OK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
            drop_graph(c);
            HIP_OK(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
            pba_status cs = enqueue_iteration(c, c->cap_stream);
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
            if (cs) { if (g) (void)hipGraphDestroy(g); return cs; }
            if (e != hipSuccess) return fail(c, PBA_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
            c->graph = g;
            HIP_OK(hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0));
            c->graph_valid = true;
        }
        for (int it = 0; it < n_iters; ++it) HIP_OK(hipGraphLaunch(c->gexec, c->stream));
    } else {
        for (int it = 0; it < n_iters; ++it)
            if ((s = enqueue_iteration(c, c->stream))) return s;
    }
    HIP_OK(hipEventRecord(c->ev1, c->stream));
    std::vector<double> lg((size_t)n_iters * kLogRow);
    HIP_OK(hipMemcpyAsync(lg.data(), c->logbuf.p, lg.size() * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    float ms = 0.f;
    HIP_OK(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    c->iterate_ms += ms;
    c->iterations += n_iters;
    bool any_fail = false;
    for (int it = 0; it < n_iters; ++it) {
        const double *r = &lg[kLogRow * (size_t)it];
        uint64_t t0, t1, i0, i1;
        std::memcpy(&t0, &r[6], 8);
        std::memcpy(&t1, &r[7], 8);
        std::memcpy(&i0, &r[8], 8);
        std::memcpy(&i1, &r[9], 8);
        if (log) {
            log[it].F = r[0];
            log[it].lambda = r[1];
            log[it].step_norm = r[2];
            log[it].n_valid = (int64_t)r[3];
            log[it].accepted = r[4] != 0.0;
            log[it].ms = (c->wall_khz > 0.0 && i1 >= i0) ? (float)((double)(i1 - i0) / c->wall_khz) : -1.0f;
        }
        if (r[5] != 0.0) any_fail = true;
        if (c->wall_khz > 0.0 && t1 >= t0) {
            c->iter_eval_ms += (double)(t1 - t0) / c->wall_khz;
            c->iter_evals += 1;
        }
    }
    if (use_lm) c->lam_carry = lg[kLogRow * (size_t)(n_iters - 1) + 1];
    if (any_fail && !use_lm) return fail(c, PBA_ENOTPD, "Gauss-Newton system not positive definite");
    return PBA_OK;
}

pba_status pba_loss_forward(pba_ctx *c, const float *delta, int32_t on_device, double *F_out, int64_t *n_valid_out)
{
    if (!c || !delta || !F_out) return fail(c, PBA_EINVAL, "null argument");
    pba_status s;
    if ((s = check_ready(c))) return s;
    HIP_OK(hipSetDevice(c->cfg.device));
    const int N = c->NP;   // pose variables
    if ((s = ensure(c, c->loss_delta, (size_t)N * 6 * 4))) return s;
    if ((s = ensure(c, c->loss_poses, (size_t)N * 12 * 8))) return s;
    if (on_device) {
        HIP_OK(hipMemcpyAsync(c->loss_delta.p, delta, (size_t)N * 24, hipMemcpyDeviceToDevice, c->stream));
    } else {
        for (int i = 0; i < 6 * N; ++i)
            if (!std::isfinite(delta[i])) return fail(c, PBA_EINVAL, "non-finite delta");
        HIP_OK(hipMemcpyAsync(c->loss_delta.p, delta, (size_t)N * 24, hipMemcpyHostToDevice, c->stream));
    }
    // X = X0 boxplus delta (the step buffer is scratch here)
    launch_delta_to_dx(P_<float>(c->loss_delta), P_<double>(c->dx), N, c->stream);
    launch_boxplus(P_<double>(c->poses), P_<double>(c->dx), nullptr, P_<double>(c->loss_poses), N, nullptr,
                   nullptr, c->stream);
    double *tot = P_<double>(c->totals) + 4;
    if ((s = run_eval(c, P_<double>(c->loss_poses), P_<double>(c->H_cand), P_<double>(c->b_cand), tot, false,
                      c->stream)))
        return s;
    double t[4];
    HIP_OK(hipMemcpyAsync(t, tot, sizeof t, hipMemcpyDeviceToHost, c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    *F_out = t[0];
    if (n_valid_out) *n_valid_out = (int64_t)t[2];
    c->loss_ready = true;
    return PBA_OK;
}

pba_status pba_loss_backward(pba_ctx *c, double grad_F, float *grad_delta, float *const *grad_intensity,
                             float *const *grad_depth, float *const *grad_normals, int32_t on_device)
{
    if (!c) return PBA_EINVAL;
    if (!std::isfinite(grad_F)) return fail(c, PBA_EINVAL, "non-finite grad_F");
    pba_status s;
    if ((s = check_ready(c))) return s;
    if (!c->loss_ready) return fail(c, PBA_ESTATE, "pba_loss_backward needs a preceding pba_loss_forward");
    if (c->cfg.storage_bf16)
        return fail(c, PBA_EINVAL, "the loss adjoint reads FP32 images: not available with BF16 storage");
    HIP_OK(hipSetDevice(c->cfg.device));
    const int N = c->NP;   // pose variables
    const int64_t tx = c->L().texels;
    const bool five = c->cfg.channels == 5;
    if ((s = ensure(c, c->g_int, (size_t)tx * 4))) return s;
    if ((s = ensure(c, c->g_dep, (size_t)tx * 4))) return s;
    if (five && (s = ensure(c, c->g_nrm, (size_t)tx * 12))) return s;
    if ((s = ensure(c, c->g_pose, (size_t)N * 24))) return s;
    // zero the gradient arenas with a fill kernel (as doubles over the byte range)
    launch_fill(P_<double>(c->g_int), (int64_t)tx / 2, 0.0, c->stream);
    launch_fill(P_<double>(c->g_dep), (int64_t)tx / 2, 0.0, c->stream);
    if (tx & 1) {
        HIP_OK(hipMemsetAsync(P_<float>(c->g_int) + tx - 1, 0, 4, c->stream));
        HIP_OK(hipMemsetAsync(P_<float>(c->g_dep) + tx - 1, 0, 4, c->stream));
    }
    if (five) {
        launch_fill(P_<double>(c->g_nrm), (int64_t)tx * 3 / 2, 0.0, c->stream);
        if ((tx * 3) & 1) HIP_OK(hipMemsetAsync(P_<float>(c->g_nrm) + 3 * tx - 1, 0, 4, c->stream));
    }
    // recompute the evaluation at X0 boxplus delta in adjoint mode
    const int ngrp = (int)c->groups.size();
    launch_pair_setup(P_<double>(c->loss_poses), P_<int2>(c->pairs_d), c->P, P_<SensorDev>(c->L().sensors_d),
                      P_<KfDev>(c->L().kfs_d), P_<PairDev>(c->pair_dev), P_<uint32_t>(c->counters), ngrp * kXcd,
                      c->stream);
    zbuffer_pass(c, P_<double>(c->loss_poses), c->stream, ctx_work(c));
    EvalArgs a = make_args(c);
    a.g_int = P_<float>(c->g_int);
    a.g_dep = P_<float>(c->g_dep);
    a.g_nrm = five ? P_<float>(c->g_nrm) : nullptr;
    a.adj_scale = grad_F;
    for (int g = 0; g < ngrp; ++g) {
        const auto &G = c->groups[g];
        a.counter = P_<uint32_t>(c->counters) + g * kXcd * kCtrStride;
        launch_eval_adjoint(a, c->cfg.channels, G.sm, G.tm, G.base, G.count, std::max(1, std::min(G.count, c->grid)),
                            c->stream);
    }
    HIP_OK(hipGetLastError());
    launch_reduce_pairs(c->partials.p, 1, P_<int32_t>(c->pitems), P_<int32_t>(c->ibeg), P_<int32_t>(c->icnt),
                        P_<PairDev>(c->pair_dev), P_<double>(c->pair_out), c->P, c->stream);
    launch_assemble(P_<double>(c->pair_out), c->P, P_<int2>(c->blk_rc), P_<int32_t>(c->blk_ptr),
                    P_<int32_t>(c->blk_ent), c->nblk, P_<int32_t>(c->bk_ptr), P_<int32_t>(c->bk_ent), N,
                    P_<double>(c->H_cand), P_<double>(c->b_cand), P_<double>(c->totals) + 4, c->stream);
    launch_pose_grad(P_<double>(c->b_cand), P_<float>(c->loss_delta), grad_F, P_<float>(c->g_pose), N, c->stream);
    HIP_OK(hipGetLastError());
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (grad_delta) HIP_OK(hipMemcpyAsync(grad_delta, c->g_pose.p, (size_t)N * 24, kind, c->stream));
    for (int k = 0; k < c->N; ++k) {   // every keyframe (pose variables may be shared)
        const size_t npx = (size_t)c->L().kfs_h[k].H * c->L().kfs_h[k].W;
        const int64_t off = c->L().kfs_h[k].off;
        if (grad_intensity && grad_intensity[k])
            HIP_OK(hipMemcpyAsync(grad_intensity[k], P_<float>(c->g_int) + off, npx * 4, kind, c->stream));
        if (grad_depth && grad_depth[k])
            HIP_OK(hipMemcpyAsync(grad_depth[k], P_<float>(c->g_dep) + off, npx * 4, kind, c->stream));
        if (five && grad_normals && grad_normals[k])
            HIP_OK(hipMemcpyAsync(grad_normals[k], P_<float>(c->g_nrm) + 3 * off, npx * 12, kind, c->stream));
    }
    HIP_OK(hipStreamSynchronize(c->stream));
    return PBA_OK;
}

pba_status pba_estimate_normals(pba_ctx *c, double radius_m, double min_px, double max_px, int32_t min_count)
{
    if (!c) return PBA_EINVAL;
    if (c->N == 0) return fail(c, PBA_ESTATE, "no keyframes loaded");
    if (c->cfg.channels != 5) return fail(c, PBA_ESTATE, "normal estimation needs 5 channels");
    if (!(radius_m > 0.0) || !(min_px >= 0.0) || !(max_px >= min_px) || max_px > 16.0 || min_count < 1)
        return fail(c, PBA_EINVAL, "bad normal-estimation parameters");
    HIP_OK(hipSetDevice(c->cfg.device));
    pba_status s;
    if (c->level != 0 || c->lv.size() > 1) {
        for (size_t l = 1; l < c->lv.size(); ++l) release_images(c->lv[l]);
        c->lv.resize(1);
        if (c->level != 0) {
            c->level = 0;
            if (c->P > 0 && (s = build_plan(c, c->src_h, c->tgt_h))) return s;
        }
    }
    ImageSet &is = c->lv[0];
    for (int k = 0; k < c->N; ++k) {
        const KfDev &f = is.kfs_h[k];
        const pba_sensor &S = is.sensors[f.sensor];
        const SensorDev &sd = is.sensors_dev_h[f.sensor];
        const double tau = S.model == PBA_PINHOLE ? c->cfg.occlusion_tau_pinhole : c->cfg.occlusion_tau_spherical;
        launch_normals(P_<float>(is.dep) + f.off, static_cast<char *>(is.att4.p) + f.off * att_bytes(c),
                       c->cfg.storage_bf16, f.H, f.W,
                       P_<double2>(is.lut64) + sd.lut_col, P_<double2>(is.lut64) + sd.lut_row,
                       S.model == PBA_SPHERICAL, radius_m * std::fabs(S.fx), min_px, max_px, tau, min_count,
                       c->stream);
    }
    HIP_OK(hipGetLastError());
    HIP_OK(hipStreamSynchronize(c->stream));
    drop_graph(c);
    c->system_valid = false;
    c->loss_ready = false;
    return PBA_OK;
}

pba_status pba_build_pairs(pba_ctx *c, double max_angle, double max_dist, double min_ratio, int32_t sequential,
                           int32_t cap, int32_t *src_out, int32_t *tgt_out, int32_t *n_out)
{
    if (!c) return PBA_EINVAL;
    if (!(max_angle >= 0.0) || !(max_dist >= 0.0) || !(min_ratio >= 0.0) || cap < 0)
        return fail(c, PBA_EINVAL, "negative threshold or capacity");
    if (c->N == 0) return fail(c, PBA_ESTATE, "no keyframes loaded");
    if (!c->poses_set) return fail(c, PBA_ESTATE, "poses not set");
    HIP_OK(hipSetDevice(c->cfg.device));
    const int N = c->N;
    std::vector<double> Xv((size_t)c->NP * 12), X((size_t)N * 12);
    HIP_OK(hipMemcpyAsync(Xv.data(), c->poses.p, Xv.size() * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    for (int k = 0; k < N; ++k)   // keyframe (platform) poses
        std::copy(Xv.begin() + 12 * (size_t)pose_var(c, k), Xv.begin() + 12 * (size_t)pose_var(c, k) + 12,
                  X.begin() + 12 * (size_t)k);
    // pose tests on the host; the candidates (and sequential links) are then evaluated together
    std::vector<int32_t> cs, ct;
    std::vector<char> close, seq;
    for (int s = 0; s < N; ++s)
        for (int t = 0; t < N; ++t) {
            if (s == t) continue;
            const double *a = &X[12 * (size_t)s], *b = &X[12 * (size_t)t];
            double tr = 0.0;
            for (int i = 0; i < 3; ++i)
                for (int k = 0; k < 3; ++k) tr += a[3 * k + i] * b[3 * k + i];   // trace(Ra^T Rb)
            const double ang = std::acos(std::min(1.0, std::max(-1.0, (tr - 1.0) / 2.0)));
            const double dx = a[9] - b[9], dy = a[10] - b[10], dz = a[11] - b[11];
            const bool cl = ang < max_angle && std::sqrt(dx * dx + dy * dy + dz * dz) < max_dist;
            const bool sq = sequential && (s - t == 1 || t - s == 1);
            if (!cl && !sq) continue;
            cs.push_back(s);
            ct.push_back(t);
            close.push_back(cl);
            seq.push_back(sq);
        }
    pba_status st;
    std::vector<int32_t> ks, kt;
    if (!cs.empty()) {
        if ((st = pba_set_pairs(c, (int32_t)cs.size(), cs.data(), ct.data()))) return st;
        if ((st = run_eval(c, P_<double>(c->poses), P_<double>(c->H_cand), P_<double>(c->b_cand),
                           P_<double>(c->totals) + 4, false, c->stream)))
            return st;
        std::vector<double> po((size_t)c->P * kPairOut);
        HIP_OK(hipMemcpyAsync(po.data(), c->pair_out.p, po.size() * 8, hipMemcpyDeviceToHost, c->stream));
        HIP_OK(hipStreamSynchronize(c->stream));
        for (size_t k = 0; k < cs.size(); ++k) {
            const double n_eval = po[k * kPairOut + 157], n_valid = po[k * kPairOut + 158];
            const bool ratio_ok = n_eval > 0.0 && n_valid >= min_ratio * n_eval;
            if (seq[k] || (close[k] && ratio_ok)) {
                ks.push_back(cs[k]);
                kt.push_back(ct[k]);
            }
        }
    }
    if ((st = pba_set_pairs(c, (int32_t)ks.size(), ks.data(), kt.data()))) return st;
    const int n = (int)ks.size();
    for (int k = 0; k < std::min(n, cap); ++k) {
        if (src_out) src_out[k] = ks[k];
        if (tgt_out) tgt_out[k] = kt[k];
    }
    if (n_out) *n_out = n;
    return PBA_OK;
}

pba_status pba_autotune(pba_ctx *c, pba_tune_point *points, int32_t max_points, int32_t *n_points)
{
    if (!c) return PBA_EINVAL;
    if (max_points < 0) return fail(c, PBA_EINVAL, "negative max_points");
    pba_status s;
    if ((s = check_ready(c))) return s;
    HIP_OK(hipSetDevice(c->cfg.device));
    const int sizes[6] = {512, 1024, 2048, 4096, 8192, 16384};
    const int mult[3] = {2, 4, 8};
    int best_px = c->items_px, best_grid = c->grid, n = 0;
    double best = 1e300;
    for (int si = 0; si < 6; ++si) {
        c->items_px = sizes[si];
        if ((s = build_plan(c, c->src_h, c->tgt_h))) return s;
        for (int gi = 0; gi < 3; ++gi) {
            c->grid = c->num_cu * mult[gi];
            double ms = 0.0;
            for (int rep = 0; rep < 2; ++rep) {   // the first run warms caches and code
                const double before = c->eval_ms;
                if ((s = run_eval(c, P_<double>(c->poses), P_<double>(c->H_cand), P_<double>(c->b_cand),
                                  P_<double>(c->totals) + 4, true, c->stream)))
                    return s;
                if ((s = accumulate_eval_time(c))) return s;
                ms = c->eval_ms - before;
            }
            if (points && n < max_points) points[n] = pba_tune_point{sizes[si], c->grid, ms};
            ++n;
            if (ms < best) { best = ms; best_px = sizes[si]; best_grid = c->grid; }
        }
    }
    c->items_px = best_px;
    c->grid = best_grid;
    if ((s = build_plan(c, c->src_h, c->tgt_h))) return s;
    drop_graph(c);
    HIP_OK(hipStreamSynchronize(c->stream));
    if (n_points) *n_points = std::min(n, max_points);
    return PBA_OK;
}

pba_status pba_build_pyramid(pba_ctx *c, int32_t n_levels)
{
    if (!c) return PBA_EINVAL;
    if (c->N == 0) return fail(c, PBA_ESTATE, "no keyframes loaded");
    if (n_levels < 1 || n_levels > 8) return fail(c, PBA_EINVAL, "n_levels %d out of range 1..8", n_levels);
    for (const pba_sensor &S : c->sensors)
        if ((S.height >> (n_levels - 1)) < 4 || (S.width >> (n_levels - 1)) < 4)
            return fail(c, PBA_EINVAL, "level %d of a %d x %d sensor would be below 4 x 4", n_levels - 1, S.height,
                        S.width);
    HIP_OK(hipSetDevice(c->cfg.device));
    for (size_t l = 1; l < c->lv.size(); ++l) release_images(c->lv[l]);
    c->lv.resize(n_levels);
    std::vector<int32_t> sensor_of(c->N);
    for (int k = 0; k < c->N; ++k) sensor_of[k] = c->lv[0].kfs_h[k].sensor;
    pba_status s;
    for (int l = 1; l < n_levels; ++l) {
        ImageSet &lo = c->lv[l - 1], &up = c->lv[l];
        up.sensors = lo.sensors;
        for (pba_sensor &S : up.sensors) {
            S.height /= 2;
            S.width /= 2;
            S.fx /= 2.0;
            S.fy /= 2.0;
            S.cx = (S.cx - 0.5) / 2.0;
            S.cy = (S.cy - 0.5) / 2.0;
        }
        if ((s = sensor_tables(c, up))) return s;
        if ((s = image_layout(c, up, sensor_of))) return s;
        const bool five = c->cfg.channels == 5;
        for (int k = 0; k < c->N; ++k) {
            const KfDev &a = lo.kfs_h[k], &b = up.kfs_h[k];
            const double tau = lo.sensors[a.sensor].model == PBA_PINHOLE ? c->cfg.occlusion_tau_pinhole
                                                                          : c->cfg.occlusion_tau_spherical;
            launch_downsample(P_<float>(lo.dep) + a.off,
                              static_cast<char *>(att_plane(c, lo)) + a.off * att_bytes(c), five ? 1 : 0,
                              c->cfg.storage_bf16, a.H, a.W, P_<float>(up.dep) + b.off,
                              static_cast<char *>(att_plane(c, up)) + b.off * att_bytes(c), b.H, b.W, tau, c->stream);
        }
        build_gate(c, up);
        HIP_OK(hipGetLastError());
    }
    HIP_OK(hipStreamSynchronize(c->stream));
    if (c->level >= n_levels) return pba_set_level(c, 0);
    return PBA_OK;
}

pba_status pba_set_level(pba_ctx *c, int32_t level)
{
    if (!c) return PBA_EINVAL;
    if (level < 0 || level >= (int)c->lv.size())
        return fail(c, PBA_EINVAL, "level %d not built (%d levels)", level, (int)c->lv.size());
    if (level == c->level) return PBA_OK;
    HIP_OK(hipSetDevice(c->cfg.device));
    drop_graph(c);
    c->level = level;
    c->system_valid = false;
    c->loss_ready = false;
    c->lam_carry = -1.0;
    pba_status s;
    if (c->P > 0 && (s = build_plan(c, c->src_h, c->tgt_h))) return s;
    HIP_OK(hipStreamSynchronize(c->stream));
    return PBA_OK;
}

pba_status pba_optimize_pyramid(pba_ctx *c, const int32_t *iters, double rel_tol, int32_t use_lm, double lambda0,
                                pba_iter_log *log, int32_t *level_of, int32_t *n_done)
{
    if (!c || !iters) return fail(c, PBA_EINVAL, "null argument");
    if (!(rel_tol >= 0.0) || (use_lm && !(lambda0 > 0.0))) return fail(c, PBA_EINVAL, "bad rel_tol or lambda0");
    pba_status s;
    if ((s = check_ready(c))) return s;
    const int nl = (int)c->lv.size();
    for (int l = 0; l < nl; ++l)
        if (iters[l] < 0) return fail(c, PBA_EINVAL, "iters[%d] < 0", l);
    int done = 0;
    for (int l = nl - 1; l >= 0; --l) {
        if ((s = pba_set_level(c, l))) return s;
        if (iters[l] == 0) continue;
        // F at the level's start: the system at the current poses
        if ((s = run_eval(c, P_<double>(c->poses), P_<double>(c->H), P_<double>(c->b), P_<double>(c->totals), false,
                          c->stream)))
            return s;
        double F_prev;
        HIP_OK(hipMemcpyAsync(&F_prev, c->totals.p, 8, hipMemcpyDeviceToHost, c->stream));
        HIP_OK(hipStreamSynchronize(c->stream));
        c->system_valid = true;
        for (int it = 0; it < iters[l]; ++it) {
            pba_iter_log row;
            if ((s = pba_iterate(c, 1, use_lm, it == 0 ? (use_lm ? lambda0 : 0.0) : 0.0, &row))) return s;
            if (log) log[done] = row;
            if (level_of) level_of[done] = l;
            ++done;
            const bool small = row.accepted && F_prev > 0.0 && (F_prev - row.F) / F_prev < rel_tol;
            if (row.accepted) F_prev = row.F;
            if (small) break;
        }
    }
    if (n_done) *n_done = done;
    return pba_set_level(c, 0);
}

pba_status pba_get_level_image(pba_ctx *c, int32_t level, int32_t kf, float *intensity, float *depth, float *normals,
                               int32_t *dims)
{
    if (!c) return PBA_EINVAL;
    if (level < 0 || level >= (int)c->lv.size())
        return fail(c, PBA_EINVAL, "level %d not built (%d levels)", level, (int)c->lv.size());
    if (kf < 0 || kf >= c->N) return fail(c, PBA_EINVAL, "keyframe %d out of range", kf);
    ImageSet &is = c->lv[level];
    const KfDev &f = is.kfs_h[kf];
    if (dims) { dims[0] = f.H; dims[1] = f.W; }
    if (!intensity && !depth && !normals) return PBA_OK;
    HIP_OK(hipSetDevice(c->cfg.device));
    const size_t npx = (size_t)f.H * f.W;
    DevBuf tmp;
    pba_status s;
    if ((s = ensure(c, tmp, npx * 5 * 4))) return s;
    float *I = P_<float>(tmp), *D = I + npx, *N = D + npx;
    const bool five = c->cfg.channels == 5;
    launch_unpack(P_<float>(is.dep) + f.off, static_cast<char *>(att_plane(c, is)) + f.off * att_bytes(c), five ? 1 : 0,
                  c->cfg.storage_bf16, (int)npx, I, D, five ? N : nullptr, c->stream);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && intensity) e = hipMemcpyAsync(intensity, I, npx * 4, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && depth) e = hipMemcpyAsync(depth, D, npx * 4, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && normals) {
        if (five) e = hipMemcpyAsync(normals, N, npx * 12, hipMemcpyDeviceToHost, c->stream);
        else std::memset(normals, 0, npx * 12);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    release(tmp);
    if (e != hipSuccess) return fail(c, PBA_EDEVICE, "pba_get_level_image: %s", hipGetErrorString(e));
    return PBA_OK;
}

pba_status pba_debug_pair(pba_ctx *c, int32_t pair, uint8_t *status, float *uv, int32_t *cell, float *residuals)
{
    if (!c) return PBA_EINVAL;
    pba_status s;
    if ((s = check_ready(c))) return s;
    if (pair < 0 || pair >= c->P) return fail(c, PBA_EINVAL, "pair %d out of range", pair);
    HIP_OK(hipSetDevice(c->cfg.device));
    // pair transforms at the current poses
    launch_pair_setup(P_<double>(c->poses), P_<int2>(c->pairs_d), c->P, P_<SensorDev>(c->L().sensors_d),
                      P_<KfDev>(c->L().kfs_d), P_<PairDev>(c->pair_dev), P_<uint32_t>(c->counters), 64, c->stream);
    zbuffer_pass(c, P_<double>(c->poses), c->stream, ctx_work(c));
    int2 pr;
    HIP_OK(hipMemcpyAsync(&pr, P_<int2>(c->pairs_d) + pair, sizeof pr, hipMemcpyDeviceToHost, c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    const KfDev &ks = c->L().kfs_h[pr.x], &kt = c->L().kfs_h[pr.y];
    const int npx = ks.H * ks.W;
    if ((s = ensure(c, c->dbg_status, npx))) return s;
    if ((s = ensure(c, c->dbg_uv, (size_t)npx * 8))) return s;
    if ((s = ensure(c, c->dbg_cell, (size_t)npx * 8))) return s;
    if ((s = ensure(c, c->dbg_res, (size_t)npx * 20))) return s;
    launch_fill(P_<double>(c->dbg_res), (int64_t)npx * 20 / 8, 0.0, c->stream);
    EvalArgs a = make_args(c);
    a.counter = P_<uint32_t>(c->counters);
    a.item_map = P_<int32_t>(c->pitems);
    a.dbg_status = P_<uint8_t>(c->dbg_status);
    a.dbg_uv = P_<float2>(c->dbg_uv);
    a.dbg_cell = P_<int2>(c->dbg_cell);
    a.dbg_res = P_<float>(c->dbg_res);
    const int sm = c->sensors[ks.sensor].model, tm = c->sensors[kt.sensor].model;
    const int base = c->pair_item_begin[pair], cnt = c->pair_item_count[pair];
    launch_eval(a, c->cfg.precision, c->cfg.channels, c->cfg.grad_mode, sm, tm, true, base, cnt,
                std::max(1, std::min(cnt, c->grid)), c->stream);
    HIP_OK(hipGetLastError());
    if (status) HIP_OK(hipMemcpyAsync(status, c->dbg_status.p, npx, hipMemcpyDeviceToHost, c->stream));
    if (uv) HIP_OK(hipMemcpyAsync(uv, c->dbg_uv.p, (size_t)npx * 8, hipMemcpyDeviceToHost, c->stream));
    if (cell) HIP_OK(hipMemcpyAsync(cell, c->dbg_cell.p, (size_t)npx * 8, hipMemcpyDeviceToHost, c->stream));
    if (residuals) HIP_OK(hipMemcpyAsync(residuals, c->dbg_res.p, (size_t)npx * 20, hipMemcpyDeviceToHost, c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    return PBA_OK;
}

pba_status pba_get_timings(pba_ctx *c, pba_timings *out, int32_t reset)
{
    if (!c || !out) return fail(c, PBA_EINVAL, "null argument");
    out->eval_ms = c->eval_ms;
    out->eval_launches = c->eval_launches;
    out->iterate_ms = c->iterate_ms;
    out->iterations = c->iterations;
    out->n_items = c->n_items;
    out->items_px = c->items_px;
    out->grid = c->grid;
    out->iter_eval_ms = c->iter_eval_ms;
    out->iter_evals = c->iter_evals;
    out->solve_n = c->chol.rows ? c->chol.n : 0;
    out->solve_steps = !c->chol.rows ? 0 : c->chol.nd ? (int32_t)c->chol.lcnt.size() : (int32_t)c->chol.rcnt.size();
    out->solve_nd = c->chol.rows && c->chol.nd ? 1 : 0;
    out->reserved = 0;
    if (reset) {
        c->eval_ms = c->iterate_ms = c->iter_eval_ms = 0.0;
        c->eval_launches = c->iterations = c->iter_evals = 0;
    }
    return PBA_OK;
}

}  // extern "C"
