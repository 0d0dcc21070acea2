// Normal estimation from depth (Sec. IV-A): the normal at u is the normal of the least-squares
// plane through the unprojected neighbours u' with |u - u'| < tau_u, tau_u inversely proportional
// to the range at u, oriented towards the observer.
//
// tau_u = clamp(radius_m |fx| / d(u), min_px, max_px) pixels (a fixed metric radius seen at range
// d); neighbours need valid depth within tau (the sensor model's occlusion threshold) of d(u);
// the fit is the eigenvector of the smallest eigenvalue of the neighbours' covariance (cyclic
// Jacobi on the 3 x 3 matrix, FP64); at least min_count points and a second eigenvalue above
// 1e-12 of the trace; oriented so that n . q_u < 0.  Pixels without a normal get 0.

#include "pba_internal.h"

namespace pba {

// Eigenvector of the smallest eigenvalue of the symmetric 3 x 3 matrix a (row-major), by cyclic
// Jacobi rotations; also the two smallest eigenvalues.
__device__ static void smallest_eigvec(double (&a)[9], double (&v)[3], double &lmin, double &lmid)
{
    double V[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    for (int sweep = 0; sweep < 12; ++sweep) {
        const double off = a[1] * a[1] + a[2] * a[2] + a[5] * a[5];
        const double dia = a[0] * a[0] + a[4] * a[4] + a[8] * a[8];
        if (!(off > 1e-34 * dia)) break;
#pragma unroll
        for (int pq = 0; pq < 3; ++pq) {
            const int p = pq == 2 ? 1 : 0, q = pq == 0 ? 1 : 2;
            const double apq = a[3 * p + q];
            if (apq == 0.0) continue;
            const double theta = (a[3 * q + q] - a[3 * p + p]) / (2.0 * apq);
            const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
            // a <- J^T a J with the rotation in the (p, q) plane
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double akp = a[3 * k + p], akq = a[3 * k + q];
                a[3 * k + p] = c * akp - s * akq;
                a[3 * k + q] = s * akp + c * akq;
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double apk = a[3 * p + k], aqk = a[3 * q + k];
                a[3 * p + k] = c * apk - s * aqk;
                a[3 * q + k] = s * apk + c * aqk;
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double vkp = V[3 * k + p], vkq = V[3 * k + q];
                V[3 * k + p] = c * vkp - s * vkq;
                V[3 * k + q] = s * vkp + c * vkq;
            }
        }
    }
    int i0 = 0;
    if (a[4] < a[3 * i0 + i0]) i0 = 1;
    if (a[8] < a[3 * i0 + i0]) i0 = 2;
    const int i1 = i0 == 0 ? 1 : 0, i2 = i0 == 2 ? 1 : 2;
    lmin = a[3 * i0 + i0];
    lmid = fmin(a[3 * i1 + i1], a[3 * i2 + i2]);
    v[0] = V[i0];
    v[1] = V[3 + i0];
    v[2] = V[6 + i0];
}

__global__ void normals_kernel(const float *__restrict__ dep, void *__restrict__ att4, int bf, int H, int W,
                               const double2 *__restrict__ lcol, const double2 *__restrict__ lrow, int spherical,
                               double scale, double min_px, double max_px, double tau, int min_count, int R)
{
    const int npx = H * W;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < npx; i += gridDim.x * blockDim.x) {
        const int r = i / W, c = i - r * W;
        const double d = (double)dep[i];
        float4 out = att_get4(att4, bf, i);
        out.y = out.z = out.w = 0.f;
        if (d > 0.0) {
            const double rad = fmin(fmax(scale / d, min_px), max_px);
            int n = 0;
            double s1[3] = {0, 0, 0}, s2[6] = {0, 0, 0, 0, 0, 0};
            for (int dy = -R; dy <= R; ++dy) {
                const int rr = r + dy;
                if (rr < 0 || rr >= H) continue;
                for (int dx = -R; dx <= R; ++dx) {
                    const int cc = c + dx;
                    if (cc < 0 || cc >= W) continue;
                    if (!(sqrt((double)(dx * dx + dy * dy)) < rad)) continue;
                    const double dn = (double)dep[rr * W + cc];
                    if (!(dn > 0.0) || !(fabs(dn - d) <= tau)) continue;
                    const double2 lc = lcol[cc], lr = lrow[rr];
                    double q0, q1, q2;
                    if (spherical) { q0 = dn * (lr.x * lc.x); q1 = dn * (lr.x * lc.y); q2 = dn * lr.y; }
                    else { q0 = dn * lc.x; q1 = dn * lr.x; q2 = dn; }
                    ++n;
                    s1[0] += q0; s1[1] += q1; s1[2] += q2;
                    s2[0] += q0 * q0; s2[1] += q0 * q1; s2[2] += q0 * q2;
                    s2[3] += q1 * q1; s2[4] += q1 * q2; s2[5] += q2 * q2;
                }
            }
            const double cn = (double)(n > 0 ? n : 1);
            const double m0 = s1[0] / cn, m1 = s1[1] / cn, m2 = s1[2] / cn;
            double A[9];
            A[0] = s2[0] / cn - m0 * m0; A[1] = s2[1] / cn - m0 * m1; A[2] = s2[2] / cn - m0 * m2;
            A[4] = s2[3] / cn - m1 * m1; A[5] = s2[4] / cn - m1 * m2; A[8] = s2[5] / cn - m2 * m2;
            A[3] = A[1]; A[6] = A[2]; A[7] = A[5];
            const double tr = A[0] + A[4] + A[8];
            double v[3], lmin, lmid;
            smallest_eigvec(A, v, lmin, lmid);
            if (n >= min_count && lmid > 1e-12 * fmax(tr, 1e-300)) {
                const double2 lc = lcol[c], lr = lrow[r];
                double q0, q1, q2;
                if (spherical) { q0 = d * (lr.x * lc.x); q1 = d * (lr.x * lc.y); q2 = d * lr.y; }
                else { q0 = d * lc.x; q1 = d * lr.x; q2 = d; }
                const double sg = v[0] * q0 + v[1] * q1 + v[2] * q2 > 0.0 ? -1.0 : 1.0;
                out.y = (float)(sg * v[0]);
                out.z = (float)(sg * v[1]);
                out.w = (float)(sg * v[2]);
            }
        }
        att_put4(att4, bf, i, out);
    }
}

void launch_normals(const float *dep, void *att4, int bf, int H, int W, const double2 *lcol, const double2 *lrow,
                    int spherical, double scale, double min_px, double max_px, double tau, int min_count,
                    hipStream_t st)
{
    const int npx = H * W;
    const int blocks = (npx + 255) / 256 < 4096 ? (npx + 255) / 256 : 4096;
    hipLaunchKernelGGL(normals_kernel, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, st, dep, att4, bf, H, W, lcol, lrow,
                       spherical, scale, min_px, max_px, tau, min_count, (int)floor(max_px));
}

}  // namespace pba
