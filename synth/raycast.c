/*
 * Seeded ray-caster for synthetic keyframes (test and benchmark inputs).
 *
 * Renders, for each keyframe, an intensity image, a depth image (pinhole:
 * distance to the image plane; spherical: range along the ray) and a normal
 * image (sensor frame, oriented towards the sensor) from a scene made of
 * textured planar rectangles plus an optional textured ground plane z = 0.
 *
 * This module only renders inputs.  It holds none of the bundle-adjustment
 * arithmetic (no warp, no sampling of keyframes, no residuals, Jacobians or
 * reductions).  Its camera code is the rendering side of the sensor
 * conventions: a pinhole pixel (col u, row v) looks along
 * ((u-cx)/fx, (v-cy)/fy, 1); a spherical pixel looks along
 * (cos el cos az, cos el sin az, sin el) with az = (u-cx)/fx, el = (v-cy)/fy.
 *
 * Noise is drawn from a counter-based generator (SplitMix64 finaliser over
 * (seed, keyframe, pixel, channel)), so output does not depend on threads.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NSIN 8

typedef struct {
    double c[3];           /* centre */
    double e1[3], e2[3];   /* unit in-plane axes */
    double n[3];           /* unit normal = e1 x e2 */
    double h1, h2;         /* half extents along e1, e2 */
    double radius;         /* bounding-sphere radius */
    double tex[NSIN][4];   /* per sinusoid: k1, k2 (cycles/m), phase, weight */
} Rect;

typedef struct {
    int model;             /* 0 pinhole, 1 spherical */
    int H, W;
    double fx, fy, cx, cy;
    double max_depth;
} Cam;

/* ---------------------------------------------------------------- rng */
static inline uint64_t mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static inline double u01(uint64_t h) { return ((h >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
static double gauss(uint64_t seed, uint64_t kf, uint64_t pix, uint64_t ch) {
    uint64_t h = mix64(seed ^ mix64(kf * 0x100000001B3ull ^ mix64(pix * 8 + ch)));
    double a = u01(h), b = u01(mix64(h));
    return sqrt(-2.0 * log(a)) * cos(6.283185307179586 * b);
}

/* ---------------------------------------------------------------- texture */
static double texture(const double t[NSIN][4], double s, double q) {
    double acc = 0.0, wsum = 0.0;
    for (int k = 0; k < NSIN; ++k) {
        acc += t[k][3] * sin(6.283185307179586 * (t[k][0] * s + t[k][1] * q) + t[k][2]);
        wsum += t[k][3];
    }
    return wsum > 0 ? 0.5 + 0.5 * acc / wsum : 0.5;
}

static inline double dot3(const double *a, const double *b) { return a[0]*b[0] + a[1]*b[1] + a[2]*b[2]; }

/* ray direction in the sensor frame (not normalised for pinhole) */
static void cam_ray(const Cam *cm, double u, double v, double d[3]) {
    if (cm->model == 0) {
        d[0] = (u - cm->cx) / cm->fx; d[1] = (v - cm->cy) / cm->fy; d[2] = 1.0;
    } else {
        double az = (u - cm->cx) / cm->fx, el = (v - cm->cy) / cm->fy;
        d[0] = cos(el) * cos(az); d[1] = cos(el) * sin(az); d[2] = sin(el);
    }
}

static void unit(double d[3]) {
    double n = sqrt(dot3(d, d));
    d[0] /= n; d[1] /= n; d[2] /= n;
}

#define TILE 16

/*
 * Render keyframes.
 *   rects[nrect], ground (0/1) with ground texture gtex.
 *   poses[nkf][12]: sensor -> world, row-major R then t.
 *   out_i/out_d: [nkf][H][W]; out_n: [nkf][H][W][3].  noise_i/noise_d: sigma.
 * Pixels with no hit within max_depth get depth 0, intensity 0, normal 0.
 */
int synth_render(const Rect *rects, int nrect, int ground, const double *gtex,
                 const Cam *cm, int nkf, const double *poses,
                 double noise_i, double noise_d, uint64_t seed, int kf_id_base,
                 float *out_i, float *out_d, float *out_n)
{
    const int H = cm->H, W = cm->W;
    const int ty = (H + TILE - 1) / TILE, tx = (W + TILE - 1) / TILE;
    const double (*gt)[4] = (const double (*)[4])gtex;
    int rc = 0;

    /* per-keyframe distance culling */
    int **near = (int **)calloc((size_t)nkf, sizeof(int *));
    int *nnear = (int *)calloc((size_t)nkf, sizeof(int));
    if (!near || !nnear) return -1;
    #pragma omp parallel for schedule(dynamic)
    for (int k = 0; k < nkf; ++k) {
        const double *o = poses + 12 * k + 9;
        int *lst = (int *)malloc(sizeof(int) * (size_t)(nrect > 0 ? nrect : 1));
        int m = 0;
        for (int r = 0; r < nrect; ++r) {
            double v[3] = {rects[r].c[0] - o[0], rects[r].c[1] - o[1], rects[r].c[2] - o[2]};
            double dist = sqrt(dot3(v, v));
            double reach = cm->model == 0 ? cm->max_depth * 3.0 : cm->max_depth;
            if (dist - rects[r].radius <= reach) lst[m++] = r;
        }
        near[k] = lst; nnear[k] = m;
    }

    const long ntiles = (long)nkf * ty * tx;
    #pragma omp parallel
    {
        int *cand = (int *)malloc(sizeof(int) * (size_t)(nrect > 0 ? nrect : 1));
        #pragma omp for schedule(dynamic, 4)
        for (long it = 0; it < ntiles; ++it) {
            const int k = (int)(it / (ty * tx));
            const int tyi = (int)((it / tx) % ty), txi = (int)(it % tx);
            const double *R = poses + 12 * k, *o = poses + 12 * k + 9;
            const int v0 = tyi * TILE, u0 = txi * TILE;
            const int v1 = v0 + TILE < H ? v0 + TILE : H, u1 = u0 + TILE < W ? u0 + TILE : W;

            /* cone around the tile: axis through its centre, half-angle to corners */
            double ax[3], axw[3];
            cam_ray(cm, 0.5 * (u0 + u1 - 1), 0.5 * (v0 + v1 - 1), ax); unit(ax);
            for (int i = 0; i < 3; ++i) axw[i] = R[3*i]*ax[0] + R[3*i+1]*ax[1] + R[3*i+2]*ax[2];
            double cosmin = 1.0;
            const double cu[6] = {u0 - 0.5, u1 - 0.5, u0 - 0.5, u1 - 0.5, 0.5 * (u0 + u1 - 1), 0.5 * (u0 + u1 - 1)};
            const double cv[6] = {v0 - 0.5, v0 - 0.5, v1 - 0.5, v1 - 0.5, v0 - 0.5, v1 - 0.5};
            for (int q = 0; q < 6; ++q) {
                double d[3]; cam_ray(cm, cu[q], cv[q], d); unit(d);
                double c = dot3(d, ax);
                if (c < cosmin) cosmin = c;
            }
            if (cosmin > 1.0) cosmin = 1.0;
            double half = acos(cosmin) * 1.05 + 2e-3;

            int nc = 0;
            for (int j = 0; j < nnear[k]; ++j) {
                const Rect *rr = &rects[near[k][j]];
                double v[3] = {rr->c[0] - o[0], rr->c[1] - o[1], rr->c[2] - o[2]};
                double dist = sqrt(dot3(v, v));
                if (dist <= rr->radius * 1.01 + 1e-6) { cand[nc++] = near[k][j]; continue; }
                double ang = acos(fmax(-1.0, fmin(1.0, dot3(v, axw) / dist)));
                double grow = asin(fmin(1.0, rr->radius / dist));
                if (ang <= half + grow) cand[nc++] = near[k][j];
            }

            for (int v = v0; v < v1; ++v) for (int u = u0; u < u1; ++u) {
                double d[3], dw[3];
                cam_ray(cm, (double)u, (double)v, d);
                for (int i = 0; i < 3; ++i) dw[i] = R[3*i]*d[0] + R[3*i+1]*d[1] + R[3*i+2]*d[2];
                double best = INFINITY, nbest[3] = {0, 0, 0}, ibest = 0.0;
                for (int j = 0; j < nc; ++j) {
                    const Rect *rr = &rects[cand[j]];
                    double den = dot3(rr->n, dw);
                    if (fabs(den) < 1e-12) continue;
                    double w[3] = {rr->c[0] - o[0], rr->c[1] - o[1], rr->c[2] - o[2]};
                    double lam = dot3(rr->n, w) / den;
                    if (!(lam > 1e-9) || lam >= best) continue;
                    double h[3] = {o[0] + lam * dw[0] - rr->c[0], o[1] + lam * dw[1] - rr->c[1],
                                   o[2] + lam * dw[2] - rr->c[2]};
                    double s = dot3(h, rr->e1), q = dot3(h, rr->e2);
                    if (fabs(s) > rr->h1 || fabs(q) > rr->h2) continue;
                    best = lam;
                    nbest[0] = rr->n[0]; nbest[1] = rr->n[1]; nbest[2] = rr->n[2];
                    ibest = texture(rr->tex, s, q);
                }
                if (ground && dw[2] < -1e-12) {
                    double lam = -o[2] / dw[2];
                    if (lam > 1e-9 && lam < best) {
                        best = lam;
                        nbest[0] = 0; nbest[1] = 0; nbest[2] = 1;
                        ibest = texture(gt, o[0] + lam * dw[0], o[1] + lam * dw[1]);
                    }
                }
                const long pix = (long)v * W + u;
                const long idx = (long)k * H * W + pix;
                double depth = 0.0;
                if (isfinite(best)) {
                    /* pinhole: lam is the z-depth (ray has unit z); spherical: unit ray, lam is range */
                    depth = best;
                    if (depth > cm->max_depth) depth = 0.0;
                }
                if (depth > 0.0) {
                    double ns[3];  /* normal into the sensor frame: R^T n */
                    for (int i = 0; i < 3; ++i) ns[i] = R[i]*nbest[0] + R[3+i]*nbest[1] + R[6+i]*nbest[2];
                    if (dot3(ns, d) > 0) { ns[0] = -ns[0]; ns[1] = -ns[1]; ns[2] = -ns[2]; }
                    const uint64_t kfid = (uint64_t)(kf_id_base + k);
                    double iv = ibest + (noise_i > 0 ? noise_i * gauss(seed, kfid, (uint64_t)pix, 0) : 0.0);
                    double dv = depth + (noise_d > 0 ? noise_d * gauss(seed, kfid, (uint64_t)pix, 1) : 0.0);
                    if (!(dv > 0.0)) dv = 0.0;
                    out_i[idx] = (float)iv;
                    out_d[idx] = (float)dv;
                    out_n[3*idx] = (float)ns[0]; out_n[3*idx+1] = (float)ns[1]; out_n[3*idx+2] = (float)ns[2];
                } else {
                    out_i[idx] = 0.f; out_d[idx] = 0.f;
                    out_n[3*idx] = 0.f; out_n[3*idx+1] = 0.f; out_n[3*idx+2] = 0.f;
                }
            }
        }
        free(cand);
    }
    for (int k = 0; k < nkf; ++k) free(near[k]);
    free(near); free(nnear);
    return rc;
}
