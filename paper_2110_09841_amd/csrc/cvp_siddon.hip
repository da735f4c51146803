// Ray-driven reference projector SiddonK (Sec. II-D): the extinction of a
// pixel is the mean, over K x K rays from the source to the centres of a
// K x K grid of equal cells on the pixel, of the line integral of mu, each
// line integral summed voxel by voxel from the exact chord lengths (Siddon's
// parametric traversal of the voxel grid, in the incremental form of
// Amanatides & Woo / Jacobs et al.).  K -> infinity gives the area average of
// the line integrals over the pixel (eq. integ), the quantity the flat-panel
// scaling of the cutting voxel projector estimates.
//
// One pixel per group of LP lanes (LP = the power of two >= min(K^2, 64));
// a lane takes rays r = lane, lane + LP, ... < K^2, and the group's sums are
// added by a butterfly in a fixed order (bitwise reproducible).  Waves stride
// over the pixel groups (a bounded grid: the work-item count of one launch
// must stay below 2^32).  The whole
// ray runs in FP64 (the vector FP64 rate of CDNA4 equals its unpacked FP32
// rate): the ray parameter of a voxel boundary near the source would lose
// most of an FP32 mantissa.  Pixels outside the detector bounding box of the
// volume's projected corners are written as 0 without tracing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "cvp_internal.h"

namespace cvp {
namespace {

#pragma clang fp contract(off)

__device__ __forceinline__ void project_point(const DevGeom &G, const ViewGeom &V, double x1, double x2,
                                              double x3, double &chi1, double &chi2)
{
    const double r1 = x1 - V.s1, r2 = x2 - V.s2, r3 = x3 - V.s3;
    const double depth = V.dx * r1 + V.dy * r2;
    chi1 = V.c1 + V.fb1 * (V.e1x * r1 + V.e1y * r2) / depth;
    chi2 = V.c2 - V.fb2 * r3 / depth;   // e2 = (0, 0, -1)
}

// Sum of mu times the chord length (in units of |dir|) along the half-line
// s + alpha dir, alpha >= 0, through the voxel grid (the volume lies between
// the source and the detector).
__device__ double trace_ray(const DevGeom &G, const float *__restrict__ vol, const double s[3],
                            const double dir[3])
{
    const int n[3] = {G.n1, G.n2, G.n3};
    const double a[3] = {G.a1, G.a2, G.a3};
    const double lo[3] = {G.x1lo, G.x2lo, G.x3lo};
    double amin = 0.0, amax = INFINITY;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        const double hi = lo[ax] + n[ax] * a[ax];
        if (dir[ax] != 0.0) {
            const double t0 = (lo[ax] - s[ax]) / dir[ax], t1 = (hi - s[ax]) / dir[ax];
            amin = fmax(amin, fmin(t0, t1));
            amax = fmin(amax, fmax(t0, t1));
        } else if (s[ax] < lo[ax] || s[ax] > hi) {
            return 0.0;
        }
    }
    if (!(amin < amax)) return 0.0;
    // first voxel: the one containing the midpoint of the first step
    int idx[3], step[3];
    double anext[3], adelta[3];
    const double amid = amin + 1e-12 * (amax - amin);
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        const double p = s[ax] + amid * dir[ax];
        int q = (int)floor((p - lo[ax]) / a[ax]);
        q = min(max(q, 0), n[ax] - 1);
        idx[ax] = q;
        if (dir[ax] > 0.0) {
            step[ax] = 1;
            anext[ax] = (lo[ax] + (q + 1) * a[ax] - s[ax]) / dir[ax];
            adelta[ax] = a[ax] / dir[ax];
        } else if (dir[ax] < 0.0) {
            step[ax] = -1;
            anext[ax] = (lo[ax] + q * a[ax] - s[ax]) / dir[ax];
            adelta[ax] = -a[ax] / dir[ax];
        } else {
            step[ax] = 0;
            anext[ax] = INFINITY;
            adelta[ax] = INFINITY;
        }
    }
    double acc = 0.0, acur = amin;
    const int maxit = G.n1 + G.n2 + G.n3 + 3;   // every step leaves a voxel: the loop always ends
    for (int it = 0; it < maxit; ++it) {
        int ax = 0;
        double an = anext[0];
        if (anext[1] < an) { an = anext[1]; ax = 1; }
        if (anext[2] < an) { an = anext[2]; ax = 2; }
        const double aend = fmin(an, amax);
        if (aend > acur)
            acc += (double)vol[((size_t)idx[2] * G.n2 + idx[1]) * G.n1 + idx[0]] * (aend - acur);
        acur = aend;
        if (acur >= amax) break;
        idx[ax] += step[ax];
        if (idx[ax] < 0 || idx[ax] >= n[ax]) break;
        anext[ax] += adelta[ax];
    }
    return acc;
}

__global__ void __launch_bounds__(kBlock)
siddon_kernel(const DevGeom G, const int K, const int LP, const float *__restrict__ vol,
              float *__restrict__ proj)
{
    // Waves step over groups of 64 / LP pixels (the whole wave takes the
    // same trip count, so the butterfly below never splits it).
    const int64_t npix = (int64_t)G.nviews * G.N * G.M;
    const int PW = kWave / LP;
    const int64_t ngroups = (npix + PW - 1) / PW;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t wave0 = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * kWaves;
    const int r0 = lane % LP;
    for (int64_t grp = wave0; grp < ngroups; grp += nwaves) {
        const int64_t pix = grp * PW + lane / LP;
        const bool live = pix < npix;
        const int64_t p = live ? pix : 0;
        const int u = (int)(p % G.M);
        const int v = (int)((p / G.M) % G.N);
        const int view = (int)(p / ((int64_t)G.M * G.N));
        const ViewGeom V = G.views[view];

        // bounding box of the volume's eight projected corners
        double cmin1 = INFINITY, cmax1 = -INFINITY, cmin2 = INFINITY, cmax2 = -INFINITY;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const double x1 = G.x1lo + ((c & 1) ? G.n1 * G.a1 : 0.0);
            const double x2 = G.x2lo + ((c & 2) ? G.n2 * G.a2 : 0.0);
            const double x3 = G.x3lo + ((c & 4) ? G.n3 * G.a3 : 0.0);
            double h1, h2;
            project_point(G, V, x1, x2, x3, h1, h2);
            cmin1 = fmin(cmin1, h1); cmax1 = fmax(cmax1, h1);
            cmin2 = fmin(cmin2, h2); cmax2 = fmax(cmax2, h2);
        }
        const bool hit = live && u + 0.5 >= cmin1 && u - 0.5 <= cmax1 && v + 0.5 >= cmin2 && v - 0.5 <= cmax2;

        double acc = 0.0;
        if (hit) {
            const double s[3] = {V.s1, V.s2, V.s3};
            const double inv = 1.0 / K;
            const int nrays = K * K;
            for (int r = r0; r < nrays; r += LP) {
                const int ra = r / K, rb = r % K;
                const double chi1 = u - 0.5 + (rb + 0.5) * inv;
                const double chi2 = v - 0.5 + (ra + 0.5) * inv;
                // ray direction at unit depth: d + (chi1 - c1)/(f/b1) e1 + (chi2 - c2)/(f/b2) e2
                const double w1 = (chi1 - V.c1) / V.fb1, w2 = (chi2 - V.c2) / V.fb2;
                const double dir[3] = {V.dx + w1 * V.e1x, V.dy + w1 * V.e1y, -w2};
                const double len = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
                acc += trace_ray(G, vol, s, dir) * len;
            }
        }
        // fixed-order butterfly over the LP lanes of the pixel
        for (int off = 1; off < LP; off <<= 1) acc += __shfl_xor(acc, off);
        if (live && r0 == 0) proj[p] = (float)(acc / ((double)K * K));
    }
}

}  // namespace

hipError_t launch_siddon(const DevGeom &g, int K, const float *vol, float *proj, hipStream_t s)
{
    const int64_t rays = (int64_t)K * K;
    int LP = 1;
    while (LP < rays && LP < kWave) LP <<= 1;
    const int64_t npix = (int64_t)g.nviews * g.N * g.M;
    const int64_t groups = (npix + (kWave / LP) - 1) / (kWave / LP);
    // a wave per pixel group, at most 2^20 workgroups (the kernel strides)
    const int64_t blocks = std::min<int64_t>((groups + kWaves - 1) / kWaves, int64_t(1) << 20);
    hipLaunchKernelGGL(siddon_kernel, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(kBlock), 0, s, g, K, LP, vol,
                       proj);
    return hipGetLastError();
}

}  // namespace cvp
