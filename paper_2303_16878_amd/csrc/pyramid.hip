// Image pyramid kernels (Sec. IV-A: every keyframe is kept at several resolutions, each level
// half the resolution of the one below; Sec. IV-C optimises coarse to fine).
//
// One level up, each 2x2 block of texels becomes one texel (an odd last row or column is
// dropped).  Depth: the block's mean if all four depths are valid and their spread is at most
// tau, else no measurement -- a block straddling a depth edge has no single surface to stand
// for.  Intensity: the mean of the four.  Normals: the mean of the four scaled to unit length.
// A texel without depth gets intensity and normal 0 (never read: source pixels need depth, and
// so does every target tap).  Means and the normalisation run in FP64 with a fixed order of
// operations and are rounded once to FP32 (or, with BF16 storage, once to BF16).

#include "pba_internal.h"

namespace pba {

__global__ void downsample_kernel(const float *__restrict__ dep, const void *__restrict__ att, int five, int bf,
                                  int H, int W, float *__restrict__ dep2, void *__restrict__ att2, int H2, int W2,
                                  double tau)
{
    const int n2 = H2 * W2;
    for (int o = blockIdx.x * blockDim.x + threadIdx.x; o < n2; o += gridDim.x * blockDim.x) {
        const int i = o / W2, j = o - i * W2;
        const int q[4] = {(2 * i) * W + 2 * j, (2 * i) * W + 2 * j + 1, (2 * i + 1) * W + 2 * j,
                          (2 * i + 1) * W + 2 * j + 1};
        double d[4];
        bool ok = true;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            d[k] = (double)dep[q[k]];
            ok = ok && d[k] > 0.0;
        }
        const double lo = fmin(fmin(d[0], d[1]), fmin(d[2], d[3]));
        const double hi = fmax(fmax(d[0], d[1]), fmax(d[2], d[3]));
        ok = ok && __dsub_rn(hi, lo) <= tau;
        const auto mean4 = [](double a, double b, double c, double e) {
            return __dmul_rn(__dadd_rn(__dadd_rn(__dadd_rn(a, b), c), e), 0.25);
        };
        dep2[o] = ok ? (float)mean4(d[0], d[1], d[2], d[3]) : kNoDepth;
        if (five) {
            float4 t[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) t[k] = att_get4(att, bf, q[k]);
            float4 r = make_float4(0.f, 0.f, 0.f, 0.f);
            if (ok) {
                r.x = (float)mean4(t[0].x, t[1].x, t[2].x, t[3].x);
                const double mx = mean4(t[0].y, t[1].y, t[2].y, t[3].y);
                const double my = mean4(t[0].z, t[1].z, t[2].z, t[3].z);
                const double mz = mean4(t[0].w, t[1].w, t[2].w, t[3].w);
                const double nn = sqrt(__dadd_rn(__dadd_rn(__dmul_rn(mx, mx), __dmul_rn(my, my)), __dmul_rn(mz, mz)));
                if (nn > 0.0) {
                    r.y = (float)__ddiv_rn(mx, nn);
                    r.z = (float)__ddiv_rn(my, nn);
                    r.w = (float)__ddiv_rn(mz, nn);
                }
            }
            att_put4(att2, bf, o, r);
        } else {
            att_put1(att2, bf, o,
                     ok ? (float)mean4(att_get1(att, bf, q[0]), att_get1(att, bf, q[1]), att_get1(att, bf, q[2]),
                                       att_get1(att, bf, q[3]))
                        : 0.f);
        }
    }
}

void launch_downsample(const float *dep, const void *att, int five, int bf, int H, int W, float *dep2, void *att2,
                       int H2, int W2, double tau, hipStream_t st)
{
    const int n2 = H2 * W2;
    const int blocks = (n2 + 255) / 256 < 4096 ? (n2 + 255) / 256 : 4096;
    hipLaunchKernelGGL(downsample_kernel, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, st, dep, att, five, bf, H, W,
                       dep2, att2, H2, W2, tau);
}

// Packed planes of one keyframe back to the caller's layout: intensity [H][W], depth [H][W]
// (0 where there is no measurement), normals [H][W][3] (may be null).
__global__ void unpack_kernel(const float *__restrict__ dep, const void *__restrict__ att, int five, int bf, int npx,
                              float *__restrict__ I, float *__restrict__ D, float *__restrict__ N)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < npx; i += gridDim.x * blockDim.x) {
        const float d = dep[i];
        D[i] = d > 0.f ? d : 0.f;
        if (five) {
            const float4 t = att_get4(att, bf, i);
            I[i] = t.x;
            if (N) { N[3 * i] = t.y; N[3 * i + 1] = t.z; N[3 * i + 2] = t.w; }
        } else {
            I[i] = att_get1(att, bf, i);
        }
    }
}

void launch_unpack(const float *dep, const void *att, int five, int bf, int npx, float *I, float *D, float *N,
                   hipStream_t st)
{
    const int blocks = (npx + 255) / 256 < 4096 ? (npx + 255) / 256 : 4096;
    hipLaunchKernelGGL(unpack_kernel, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, st, dep, att, five, bf, npx, I, D,
                       N);
}

}  // namespace pba
