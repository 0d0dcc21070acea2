/*
 * Plain FP64 CPU oracle of the photometric bundle-adjustment evaluation.
 * TEST INFRASTRUCTURE ONLY: the product path never links or calls this file.
 *
 * For one ordered pair (s, t) -- the paper's <i, j>: the cloud of image i
 * (source s) is warped into image j (target t) -- it computes, pixel by pixel,
 * the multi-cue residuals, their robust weight and the Jacobians with respect
 * to both poses, and accumulates the 12x12 block [dx_s; dx_t] of
 * H = sum w J^T Omega J, the 12-vector b = sum w J^T Omega e, the loss
 * F = sum rho(chi^2) and the counts.  It follows the paper step by step:
 *   unprojection pi^-1 and the projections pi_p / pi_s      Sec. III (Basics)
 *   warp u' = pi(R_j^T (R_i pi^-1(u,d) + t_i - t_j))          Sec. IV-C, Eq. (uprime)
 *   multi-cue robust error F                                  Sec. IV-C, Eq. (total-error-multicue)
 *   sensor offset p_u, p_bar                                  Supplementary, point definitions
 *   dp_bar/dx_i, dp_bar/dx_j                                  Supplementary, point Jacobians
 *   pinhole / spherical projective Jacobians                 Supplementary
 *   central-difference image Jacobians                        Supplementary
 *   intensity, depth, range and normal cue maps and their Jacobians
 *   full Jacobians J_i, J_j                                   Supplementary, last equations
 * The paper's skew operator is written here as skewp(v): skewp(v) w = w x v,
 * the convention under which the supplementary formulas are exact.  The
 * source-normal Jacobian is taken as 2 R_o^T R_j^T R_i skewp(R_o n_u) (the
 * printed formula has R_j for R_j^T and R_o skewp(n_u) for skewp(R_o n_u)).
 *
 * Built with -O2 -ffp-contract=off: no fused multiply-adds, IEEE rounding.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t model, H, W, pad;   /* model: 0 pinhole, 1 spherical */
    double fx, fy, cx, cy, dmin, dmax;
    double Ro[9], to[3];        /* sensor -> platform offset */
} OrcSensor;

typedef struct {
    int32_t channels;           /* 2: intensity + depth; 5: + normal xyz */
    int32_t grad_mode;          /* 0: central differences blended bilinearly; 1: exact bilinear slope */
    double omega[3];            /* information of intensity, depth, normal */
    double huber;               /* <= 0: plain squares */
    double occ_tau;             /* occlusion gate on |e_depth| for this pair's target */
    int32_t zbuffer;            /* 1: also the source z-buffer test (occlusion by the pair's own points) */
    int32_t pad;
} OrcParams;

typedef struct {
    double H[144];              /* 12x12 row-major, variables [dx_s (6); dx_t (6)] */
    double b[12];
    double F;
    int64_t n_eval, n_valid;
    double babs[12];            /* sum of |w Omega J e| per component: the scale b cancels against */
} OrcPairOut;

/* per-pixel status codes */
enum { ST_VALID = 0, ST_NODEPTH = 1, ST_NOPROJ = 2, ST_OUTSIDE = 3, ST_BADTAP = 4, ST_OCCLUDED = 5,
       ST_SKIPPED = 6, ST_ZOCCLUDED = 7 };

/* ---------------------------------------------------------------- 3x3 helpers (row-major) */
static void matmul3(const double *A, const double *B, double *C) {
    double T[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            T[3*i+j] = A[3*i]*B[j] + A[3*i+1]*B[3+j] + A[3*i+2]*B[6+j];
    memcpy(C, T, sizeof T);
}
static void transpose3(const double *A, double *T) {
    for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) T[3*j+i] = A[3*i+j];
}
static void matvec3(const double *A, const double *v, double *o) {
    double r[3];
    for (int i = 0; i < 3; ++i) r[i] = A[3*i]*v[0] + A[3*i+1]*v[1] + A[3*i+2]*v[2];
    o[0] = r[0]; o[1] = r[1]; o[2] = r[2];
}
/* the paper's skew: skewp(v) w = w x v */
static void skewp(const double *v, double *S) {
    S[0] = 0;     S[1] = v[2];  S[2] = -v[1];
    S[3] = -v[2]; S[4] = 0;     S[5] = v[0];
    S[6] = v[1];  S[7] = -v[0]; S[8] = 0;
}

static int depth_ok(double d, const OrcSensor *s) {
    return isfinite(d) && d > 0.0 && d >= s->dmin && d <= s->dmax;
}

/* inverse projection pi^-1(u, d) in the sensor frame (Sec. III) */
static void unproject(const OrcSensor *s, double col, double row, double d, double *q) {
    if (s->model == 0) {
        q[0] = d * (col - s->cx) / s->fx;
        q[1] = d * (row - s->cy) / s->fy;
        q[2] = d;
    } else {
        double az = (col - s->cx) / s->fx, el = (row - s->cy) / s->fy;
        q[0] = d * cos(el) * cos(az);
        q[1] = d * cos(el) * sin(az);
        q[2] = d * sin(el);
    }
}

/* projection pi(p) (Sec. III, Eqs. pinhole-projection / spherical-projection).
 * Returns 0 if the point cannot be projected (behind / too close). */
static int project(const OrcSensor *s, const double *p, double *uv) {
    if (s->model == 0) {
        if (!(p[2] >= s->dmin)) return 0;
        double v0 = s->fx * p[0] + s->cx * p[2];
        double v1 = s->fy * p[1] + s->cy * p[2];
        double v2 = p[2];
        uv[0] = v0 / v2;
        uv[1] = v1 / v2;
    } else {
        double rho = sqrt(p[0]*p[0] + p[1]*p[1]);
        double rng = sqrt(p[0]*p[0] + p[1]*p[1] + p[2]*p[2]);
        if (!(rho > 0.0) || !(rng >= s->dmin)) return 0;
        uv[0] = s->fx * atan2(p[1], p[0]) + s->cx;
        uv[1] = s->fy * atan2(p[2], rho) + s->cy;
    }
    return 1;
}

static inline double px(const float *img, int W, int r, int c) { return (double)img[(int64_t)r * W + c]; }

/* p_bar of source pixel (c, r) at depth d in the target sensor frame:
 * p_u = R_os pi_s^-1(u, d) + t_os, y = R_j^T (R_i p_u + t_i - t_j), p_bar = R_ot^T (y - t_ot). */
static void warp_pixel(const OrcSensor *ss, const OrcSensor *st, const double *Xs, const double *Xt, int c, int r,
                       double d, double *pu, double *y, double *pbar)
{
    const double *Ri = Xs, *ti = Xs + 9, *Rj = Xt, *tj = Xt + 9;
    double q[3], w3[3], ym[3], RjT[9], RotT[9];
    unproject(ss, (double)c, (double)r, d, q);
    matvec3(ss->Ro, q, pu);
    for (int k = 0; k < 3; ++k) pu[k] += ss->to[k];
    matvec3(Ri, pu, w3);
    for (int k = 0; k < 3; ++k) w3[k] += ti[k] - tj[k];
    transpose3(Rj, RjT);
    matvec3(RjT, w3, y);
    for (int k = 0; k < 3; ++k) ym[k] = y[k] - st->to[k];
    transpose3(st->Ro, RotT);
    matvec3(RotT, ym, pbar);
}

/* Source z-buffer of one pair (the z-buffer occlusion variant): for every target cell, the
 * smallest predicted depth zeta^d (p_bar_z for a pinhole target, |p_bar| for a spherical one),
 * rounded to FP32, over the pair's source points with valid depth that project with their
 * integer cell floor(u') inside the evaluated region [1, W-3] x [1, H-3]; +inf where none lands.
 * Z has Ht * Wt floats. */
void orc_zbuffer(const OrcSensor *ss, const float *Ds, const OrcSensor *st, const double *Xs, const double *Xt,
                 float *Z)
{
    const int Ht = st->H, Wt = st->W;
    for (int64_t k = 0; k < (int64_t)Ht * Wt; ++k) Z[k] = INFINITY;
    for (int r = 0; r < ss->H; ++r) for (int c = 0; c < ss->W; ++c) {
        const double d = px(Ds, ss->W, r, c);
        if (!depth_ok(d, ss)) continue;
        double pu[3], y[3], pbar[3], uv[2];
        warp_pixel(ss, st, Xs, Xt, c, r, d, pu, y, pbar);
        if (!project(st, pbar, uv)) continue;
        const double fx0 = floor(uv[0]), fy0 = floor(uv[1]);
        if (!(fx0 >= 1.0 && fx0 <= Wt - 3.0 && fy0 >= 1.0 && fy0 <= Ht - 3.0)) continue;
        const double zeta = st->model == 0 ? pbar[2] : sqrt(pbar[0]*pbar[0] + pbar[1]*pbar[1] + pbar[2]*pbar[2]);
        const int64_t cell = (int64_t)fy0 * Wt + (int64_t)fx0;
        const float zf = (float)zeta;
        if (zf < Z[cell]) Z[cell] = zf;
    }
}

/* projective Jacobian d pi / d p (2x3, row-major), Supplementary */
static void proj_jacobian(const OrcSensor *s, const double *p, double *P) {
    if (s->model == 0) {
        const double K[9] = {s->fx, 0, s->cx, 0, s->fy, s->cy, 0, 0, 1};
        double v[3];
        matvec3(K, p, v);
        const double iz2 = 1.0 / (v[2] * v[2]);
        const double A[6] = {v[2] * iz2, 0, -v[0] * iz2, 0, v[2] * iz2, -v[1] * iz2};
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 3; ++j)
                P[3*i+j] = A[3*i]*K[j] + A[3*i+1]*K[3+j] + A[3*i+2]*K[6+j];
    } else {
        const double x = p[0], y = p[1], z = p[2];
        const double r2 = x*x + y*y, rho = sqrt(r2), n2 = x*x + y*y + z*z;
        const double Psi[9] = {-y / r2, x / r2, 0,
                               -x * z / rho / n2, -y * z / rho / n2, rho / n2,
                               0, 0, 0};
        const double K12[6] = {s->fx, 0, s->cx, 0, s->fy, s->cy};
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 3; ++j)
                P[3*i+j] = K12[3*i]*Psi[j] + K12[3*i+1]*Psi[3+j] + K12[3*i+2]*Psi[6+j];
    }
}

static double huber_rho(double chi2, double delta, double *w) {
    if (!(delta > 0)) { *w = 1.0; return chi2; }
    double e = sqrt(chi2);
    if (e <= delta) { *w = 1.0; return chi2; }
    *w = delta / e;
    return 2.0 * delta * e - delta * delta;
}


/*
 * Evaluate one ordered pair.  Images are row-major [H][W] (normals [H][W][3]).
 * Xs, Xt: platform -> world poses (R row-major, then t).
 * force_valid / force_cell (both NULL or both set): use exactly the given
 * per-source-pixel validity and integer cell (x0, y0) instead of deciding
 * them here ("mask-forced" mode, for comparing sums on identical
 * correspondences).
 * Optional per-pixel outputs: status (uint8), uv (2 doubles), res (5 doubles) and
 * margin (1 double: min over the stencil taps of occ_tau - |depth_tap - zeta^d|,
 * written for pixels that reach the occlusion test) and imgjac (10 doubles: the image
 * Jacobian g_c = [dI/dcol, dI/drow] of each channel at u', written for valid pixels).
 */
/* Gradients of F with respect to the images (loss adjoint), accumulated when non-NULL:
 * source and target intensity [H][W], depth [H][W], normals [H][W][3].  The masks, the
 * integer cells and the occlusion decisions are held fixed; F is then a smooth function
 * of the image values through the bilinear samples V^c, the source intensity and normal,
 * and the source depth through the warped point p_bar. */
typedef struct {
    double *gIs, *gDs, *gNs, *gIt, *gDt, *gNt;
} OrcImageGrad;

int orc_eval_pair_grad(const OrcSensor *ss, const float *Is, const float *Ds, const float *Ns,
                       const OrcSensor *st, const float *It, const float *Dt, const float *Nt,
                       const double *Xs, const double *Xt, const OrcParams *prm,
                       const uint8_t *force_valid, const int32_t *force_cell,
                       OrcPairOut *out, uint8_t *status_out, double *uv_out, double *res_out,
                       double *margin_out, double *imgjac_out, const OrcImageGrad *ig);

int orc_eval_pair(const OrcSensor *ss, const float *Is, const float *Ds, const float *Ns,
                  const OrcSensor *st, const float *It, const float *Dt, const float *Nt,
                  const double *Xs, const double *Xt, const OrcParams *prm,
                  const uint8_t *force_valid, const int32_t *force_cell,
                  OrcPairOut *out, uint8_t *status_out, double *uv_out, double *res_out,
                  double *margin_out)
{
    return orc_eval_pair_grad(ss, Is, Ds, Ns, st, It, Dt, Nt, Xs, Xt, prm, force_valid, force_cell, out,
                              status_out, uv_out, res_out, margin_out, NULL, NULL);
}

int orc_eval_pair_grad(const OrcSensor *ss, const float *Is, const float *Ds, const float *Ns,
                       const OrcSensor *st, const float *It, const float *Dt, const float *Nt,
                       const double *Xs, const double *Xt, const OrcParams *prm,
                       const uint8_t *force_valid, const int32_t *force_cell,
                       OrcPairOut *out, uint8_t *status_out, double *uv_out, double *res_out,
                       double *margin_out, double *imgjac_out, const OrcImageGrad *ig)
{
    const int C = prm->channels;
    const int Hs = ss->H, Ws = ss->W, Ht = st->H, Wt = st->W;
    memset(out, 0, sizeof *out);

    float *Z = NULL;   /* the pair's source z-buffer (z-buffer occlusion variant) */
    if (prm->zbuffer && !force_valid) {
        Z = (float *)malloc(sizeof(float) * (size_t)Ht * Wt);
        if (!Z) return -4;
        orc_zbuffer(ss, Ds, st, Xs, Xt, Z);
    }
    const double *Ri = Xs, *ti = Xs + 9, *Rj = Xt, *tj = Xt + 9;
    double RjT[9], RjTRi[9], RotT[9], M_RotRjRi[9];
    transpose3(Rj, RjT);
    matmul3(RjT, Ri, RjTRi);                 /* R_j^T R_i */
    transpose3(st->Ro, RotT);
    matmul3(RotT, RjTRi, M_RotRjRi);         /* R_o^T R_j^T R_i (target offset) */

    for (int r = 0; r < Hs; ++r) for (int c = 0; c < Ws; ++c) {
        const int64_t pix = (int64_t)r * Ws + c;
        uint8_t status = ST_VALID;
        if (status_out) status_out[pix] = ST_NODEPTH;
        if (uv_out) { uv_out[2*pix] = NAN; uv_out[2*pix+1] = NAN; }
        if (res_out) for (int k = 0; k < 5; ++k) res_out[5*pix+k] = NAN;
        if (margin_out) margin_out[pix] = NAN;
        if (imgjac_out) for (int k = 0; k < 10; ++k) imgjac_out[10*pix+k] = NAN;

        const double d = px(Ds, Ws, r, c);
        if (!depth_ok(d, ss)) continue;
        out->n_eval++;
        if (force_valid && !force_valid[pix]) { if (status_out) status_out[pix] = ST_SKIPPED; continue; }

        /* p_u = R_o pi^-1(u, d) + t_o (source offset); y = R_j^T (R_i p_u + t_i - t_j);
         * p_bar = R_o^T (y - t_o) (target offset) */
        double pu[3], y[3], pbar[3];
        warp_pixel(ss, st, Xs, Xt, c, r, d, pu, y, pbar);

        double uv[2];
        int x0, y0;
        if (!project(st, pbar, uv)) {
            if (force_valid) return -2;     /* a forced correspondence must project */
            status = ST_NOPROJ;
            goto done;
        }
        if (uv_out) { uv_out[2*pix] = uv[0]; uv_out[2*pix+1] = uv[1]; }
        if (force_cell) {
            x0 = force_cell[2*pix]; y0 = force_cell[2*pix+1];
            if (x0 < 1 || x0 > Wt - 3 || y0 < 1 || y0 > Ht - 3) return -3;
        } else {
            double fx0 = floor(uv[0]), fy0 = floor(uv[1]);
            if (!(fx0 >= 1.0 && fx0 <= Wt - 3.0 && fy0 >= 1.0 && fy0 <= Ht - 3.0)) { status = ST_OUTSIDE; goto done; }
            x0 = (int)fx0; y0 = (int)fy0;
            /* the 12 taps used by the bilinear blend of central differences */
            const int tr[12] = {y0, y0, y0, y0, y0+1, y0+1, y0+1, y0+1, y0-1, y0-1, y0+2, y0+2};
            const int tc[12] = {x0-1, x0, x0+1, x0+2, x0-1, x0, x0+1, x0+2, x0, x0+1, x0, x0+1};
            int ok = 1;
            for (int k = 0; k < 12; ++k) ok &= depth_ok(px(Dt, Wt, tr[k], tc[k]), st);
            if (!ok) { status = ST_BADTAP; goto done; }
        }
        {
            const double a = uv[0] - x0, bb = uv[1] - y0;
            /* sample every channel: value and image Jacobian g = [dI/dcol, dI/drow] at u' */
            double V[5], G[5][2];
            for (int ch = 0; ch < C; ++ch) {
                const float *img; int stride, off;
                if (ch == 0) { img = It; stride = 1; off = 0; }
                else if (ch == 1) { img = Dt; stride = 1; off = 0; }
                else { img = Nt; stride = 3; off = ch - 2; }
#define T(rr, cc) ((double)img[((int64_t)(rr) * Wt + (cc)) * stride + off])
                const double I00 = T(y0, x0), I01 = T(y0, x0+1), I10 = T(y0+1, x0), I11 = T(y0+1, x0+1);
                V[ch] = (1-bb) * ((1-a) * I00 + a * I01) + bb * ((1-a) * I10 + a * I11);
                if (prm->grad_mode == 0) {
                    /* central differences at each of the 4 taps, blended with the bilinear weights */
                    double gc00 = 0.5 * (T(y0, x0+1) - T(y0, x0-1));
                    double gc01 = 0.5 * (T(y0, x0+2) - T(y0, x0));
                    double gc10 = 0.5 * (T(y0+1, x0+1) - T(y0+1, x0-1));
                    double gc11 = 0.5 * (T(y0+1, x0+2) - T(y0+1, x0));
                    double gr00 = 0.5 * (T(y0+1, x0) - T(y0-1, x0));
                    double gr01 = 0.5 * (T(y0+1, x0+1) - T(y0-1, x0+1));
                    double gr10 = 0.5 * (T(y0+2, x0) - T(y0, x0));
                    double gr11 = 0.5 * (T(y0+2, x0+1) - T(y0, x0+1));
                    G[ch][0] = (1-bb) * ((1-a) * gc00 + a * gc01) + bb * ((1-a) * gc10 + a * gc11);
                    G[ch][1] = (1-bb) * ((1-a) * gr00 + a * gr01) + bb * ((1-a) * gr10 + a * gr11);
                } else {
                    /* slope of the bilinear interpolant itself */
                    G[ch][0] = (1-bb) * (I01 - I00) + bb * (I11 - I10);
                    G[ch][1] = (1-a) * (I10 - I00) + a * (I11 - I01);
                }
#undef T
            }

            /* cue maps zeta^c and residuals e^c = zeta^c - I_j^c(u') */
            double zeta[5], e[5];
            zeta[0] = px(Is, Ws, r, c);
            const double range = sqrt(pbar[0]*pbar[0] + pbar[1]*pbar[1] + pbar[2]*pbar[2]);
            zeta[1] = st->model == 0 ? pbar[2] : range;
            double nrot[3] = {0, 0, 0}, Ron[3] = {0, 0, 0};
            if (C == 5) {
                const double n_u[3] = {Ns[3*pix], Ns[3*pix+1], Ns[3*pix+2]};
                double RoRo[9];
                matvec3(ss->Ro, n_u, Ron);                 /* R_o n_u (source offset) */
                matmul3(M_RotRjRi, ss->Ro, RoRo);
                matvec3(RoRo, n_u, nrot);                  /* R_o^T R_j^T R_i R_o n_u */
                zeta[2] = nrot[0]; zeta[3] = nrot[1]; zeta[4] = nrot[2];
            }
            for (int ch = 0; ch < C; ++ch) e[ch] = zeta[ch] - V[ch];
            /* occlusion suppression (Sec. IV-C): every target sample the point uses -- the 12
             * stencil taps -- must lie on the surface the point lands on, i.e. its depth must be
             * within occ_tau of the predicted depth zeta^d.  This implies |e^d| <= occ_tau. */
            if (!force_valid) {
                const int tr[12] = {y0, y0, y0, y0, y0+1, y0+1, y0+1, y0+1, y0-1, y0-1, y0+2, y0+2};
                const int tc[12] = {x0-1, x0, x0+1, x0+2, x0-1, x0, x0+1, x0+2, x0, x0+1, x0, x0+1};
                int vis = 1;
                double margin = INFINITY;
                for (int k = 0; k < 12; ++k) {
                    const double m = prm->occ_tau - fabs(px(Dt, Wt, tr[k], tc[k]) - zeta[1]);
                    vis &= m >= 0.0;
                    if (m < margin) margin = m;
                }
                if (margin_out) margin_out[pix] = margin;
                if (!vis) { status = ST_OCCLUDED; goto done; }
                /* z-buffer variant: no more than occ_tau behind the nearest of the pair's own
                 * points landing in the same cell (both depths as FP32, compared in FP64) */
                if (Z && (double)(float)zeta[1] - (double)Z[(int64_t)y0 * Wt + x0] > prm->occ_tau) {
                    status = ST_ZOCCLUDED;
                    goto done;
                }
            }
            if (res_out) for (int ch = 0; ch < C; ++ch) res_out[5*pix+ch] = e[ch];
            if (imgjac_out) for (int ch = 0; ch < C; ++ch) {
                imgjac_out[10*pix+2*ch] = G[ch][0];
                imgjac_out[10*pix+2*ch+1] = G[ch][1];
            }

            double chi2 = prm->omega[0] * e[0] * e[0] + prm->omega[1] * e[1] * e[1];
            for (int ch = 2; ch < C; ++ch) chi2 += prm->omega[2] * e[ch] * e[ch];
            double wgt;
            const double rho = huber_rho(chi2, prm->huber, &wgt);

            /* dp_bar/dx_i = R_o^T R_j^T R_i [I  2 skewp(p_u)],  dp_bar/dx_j = -R_o^T [I  2 skewp(y)] */
            double Ms[18], Mt[18], Sp[9], Sy[9], L[9];
            skewp(pu, Sp);
            matmul3(M_RotRjRi, Sp, L);
            for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) {
                Ms[6*i+j] = M_RotRjRi[3*i+j];
                Ms[6*i+3+j] = 2.0 * L[3*i+j];
            }
            skewp(y, Sy);
            matmul3(RotT, Sy, L);
            for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) {
                Mt[6*i+j] = -RotT[3*i+j];
                Mt[6*i+3+j] = -2.0 * L[3*i+j];
            }
            double P[6];
            proj_jacobian(st, pbar, P);
            double PMs[12], PMt[12];   /* (d pi / d p_bar)(d p_bar / d x) : 2x6 */
            for (int i = 0; i < 2; ++i) for (int j = 0; j < 6; ++j) {
                PMs[6*i+j] = P[3*i]*Ms[j] + P[3*i+1]*Ms[6+j] + P[3*i+2]*Ms[12+j];
                PMt[6*i+j] = P[3*i]*Mt[j] + P[3*i+1]*Mt[6+j] + P[3*i+2]*Mt[12+j];
            }
            /* d zeta^c / d x for both poses */
            double Zs[5][6], Zt[5][6];
            memset(Zs, 0, sizeof Zs); memset(Zt, 0, sizeof Zt);
            {
                double dz[3];
                if (st->model == 0) { dz[0] = 0; dz[1] = 0; dz[2] = 1; }
                else { dz[0] = pbar[0] / range; dz[1] = pbar[1] / range; dz[2] = pbar[2] / range; }
                for (int j = 0; j < 6; ++j) {
                    Zs[1][j] = dz[0]*Ms[j] + dz[1]*Ms[6+j] + dz[2]*Ms[12+j];
                    Zt[1][j] = dz[0]*Mt[j] + dz[1]*Mt[6+j] + dz[2]*Mt[12+j];
                }
            }
            if (C == 5) {
                double Sn[9], A[9], mr[3];
                skewp(Ron, Sn);
                matmul3(M_RotRjRi, Sn, A);           /* R_o^T R_j^T R_i skewp(R_o n_u) */
                matvec3(RjTRi, Ron, mr);             /* R_j^T R_i R_o n_u */
                double Sm[9], B[9];
                skewp(mr, Sm);
                matmul3(RotT, Sm, B);                /* R_o^T skewp(R_j^T R_i R_o n_u) */
                for (int k = 0; k < 3; ++k) for (int j = 0; j < 3; ++j) {
                    Zs[2+k][3+j] = 2.0 * A[3*k+j];
                    Zt[2+k][3+j] = -2.0 * B[3*k+j];
                }
            }
            /* J^c = d zeta^c/dx - g_c^T (d pi/d p_bar)(d p_bar/d x), accumulate */
            for (int ch = 0; ch < C; ++ch) {
                double J[12];
                for (int j = 0; j < 6; ++j) {
                    J[j]     = Zs[ch][j] - (G[ch][0] * PMs[j] + G[ch][1] * PMs[6+j]);
                    J[6 + j] = Zt[ch][j] - (G[ch][0] * PMt[j] + G[ch][1] * PMt[6+j]);
                }
                const double om = wgt * prm->omega[ch < 2 ? ch : 2];
                for (int i = 0; i < 12; ++i) {
                    for (int j = 0; j < 12; ++j) out->H[12*i+j] += om * J[i] * J[j];
                    out->b[i] += om * J[i] * e[ch];
                    out->babs[i] += fabs(om * J[i] * e[ch]);
                }
            }
            out->F += rho;
            out->n_valid++;

            if (ig) {
                /* dF/de^c = 2 w Omega^c e^c */
                double k[5];
                for (int ch = 0; ch < C; ++ch) k[ch] = 2.0 * wgt * prm->omega[ch < 2 ? ch : 2] * e[ch];
                /* target channels: e^c = zeta^c - V^c, V^c = sum of bilinear weights x taps */
                const double wt[4] = {(1-a) * (1-bb), a * (1-bb), (1-a) * bb, a * bb};
                const int64_t ti[4] = {(int64_t)y0 * Wt + x0, (int64_t)y0 * Wt + x0 + 1,
                                       (int64_t)(y0+1) * Wt + x0, (int64_t)(y0+1) * Wt + x0 + 1};
                for (int q = 0; q < 4; ++q) {
                    if (ig->gIt) ig->gIt[ti[q]] -= k[0] * wt[q];
                    if (ig->gDt) ig->gDt[ti[q]] -= k[1] * wt[q];
                    if (ig->gNt) for (int ch = 2; ch < C; ++ch) ig->gNt[3*ti[q] + ch - 2] -= k[ch] * wt[q];
                }
                /* source intensity: e^g = I_s(u) - V^g */
                if (ig->gIs) ig->gIs[pix] += k[0];
                /* source normal: e^n = R_ot^T R_t^T R_s R_os n_u - V^n */
                if (ig->gNs && C == 5) {
                    double RR[9];
                    matmul3(M_RotRjRi, ss->Ro, RR);
                    for (int j = 0; j < 3; ++j)
                        ig->gNs[3*pix + j] += k[2] * RR[j] + k[3] * RR[3+j] + k[4] * RR[6+j];
                }
                /* source depth: p_bar moves along R_ot^T R_t^T R_s R_os ray(u) per unit of d, and
                 * every e^c depends on p_bar through zeta^c (depth/range) and through u' = pi(p_bar) */
                if (ig->gDs) {
                    double ray[3], RR[9], dp[3];
                    unproject(ss, (double)c, (double)r, 1.0, ray);
                    matmul3(M_RotRjRi, ss->Ro, RR);
                    matvec3(RR, ray, dp);
                    double dz[3];
                    if (st->model == 0) { dz[0] = 0; dz[1] = 0; dz[2] = 1; }
                    else { dz[0] = pbar[0] / range; dz[1] = pbar[1] / range; dz[2] = pbar[2] / range; }
                    double g = 0.0;
                    for (int ch = 0; ch < C; ++ch) {
                        double ac[3];
                        for (int j = 0; j < 3; ++j) ac[j] = -(G[ch][0] * P[j] + G[ch][1] * P[3+j]);
                        if (ch == 1) for (int j = 0; j < 3; ++j) ac[j] += dz[j];
                        g += k[ch] * (ac[0] * dp[0] + ac[1] * dp[1] + ac[2] * dp[2]);
                    }
                    ig->gDs[pix] += g;
                }
            }
        }
done:
        if (status_out) status_out[pix] = status;
    }
    free(Z);
    return 0;
}

/* Evaluate many pairs (OpenMP over pairs; each pair's sums are independent). */
typedef struct {
    const float *I, *D, *N;
    int32_t sensor, pad;
} OrcFrame;

int orc_eval_pairs(const OrcSensor *sensors, const OrcFrame *frames, const double *poses,
                   int npairs, const int32_t *src, const int32_t *tgt, const OrcParams *prm_pinhole,
                   const OrcParams *prm_spherical, OrcPairOut *outs)
{
    int err = 0;
    #pragma omp parallel for schedule(dynamic, 1) reduction(|: err)
    for (int p = 0; p < npairs; ++p) {
        const OrcFrame *fs = &frames[src[p]], *ft = &frames[tgt[p]];
        const OrcSensor *ss = &sensors[fs->sensor], *st = &sensors[ft->sensor];
        const OrcParams *prm = st->model == 0 ? prm_pinhole : prm_spherical;
        int rc = orc_eval_pair(ss, fs->I, fs->D, fs->N, st, ft->I, ft->D, ft->N,
                               poses + 12 * (int64_t)src[p], poses + 12 * (int64_t)tgt[p], prm,
                               NULL, NULL, &outs[p], NULL, NULL, NULL, NULL);
        if (rc) err |= 1;
    }
    return err ? -1 : 0;
}
