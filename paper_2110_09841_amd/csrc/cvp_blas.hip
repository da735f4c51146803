// Vector kernels of CGLS on the GPU: FP64-accumulated dot products with a
// fixed-order two-stage reduction, fused axpy updates, and the scalar
// recurrences kept on the device (no host round trip between iterations, so
// a run of iterations can be captured in a HIP graph).  All of them are
// HBM-bound streaming kernels: float4 accesses, grid-stride loops.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "cvp_internal.h"

namespace cvp {
namespace {

constexpr int kRedBlocks = kCglsPartials;   // partial sums per reduction
constexpr int kRedThreads = 256;

__device__ __forceinline__ double block_sum(double v, double *sh)
{
    const int tid = threadIdx.x;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if ((tid & 63) == 0) sh[tid >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (tid == 0)
        for (int w = 0; w < kRedThreads / 64; ++w) s += sh[w];
    return s;
}

// partial[b] = sum over this block's elements of a[i] * c[i] (FP64)
__device__ __forceinline__ bool stopped(const double *stop) { return stop && *stop != 0.0; }

__global__ void __launch_bounds__(kRedThreads)
dot_partials(const float *__restrict__ a, const float *__restrict__ c, int64_t n,
             double *__restrict__ partial, const double *__restrict__ stop)
{
    if (stopped(stop)) return;
    __shared__ double sh[kRedThreads / 64];
    double acc = 0.0;
    const int64_t n4 = n / 4;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const bool vec = ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(c)) & 15) == 0;
    int64_t tail0 = 0;
    if (vec) {
        const float4 *a4 = reinterpret_cast<const float4 *>(a);
        const float4 *c4 = reinterpret_cast<const float4 *>(c);
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) {
            const float4 x = a4[i], y = c4[i];
            acc += (double)x.x * y.x + (double)x.y * y.y + (double)x.z * y.z + (double)x.w * y.w;
        }
        tail0 = n4 * 4;
    }
    for (int64_t i = tail0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        acc += (double)a[i] * c[i];
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

enum : int { kFinStart = 0, kFinQQ = 1, kFinGamma = 2, kFinRR = 3, kFinDot = 4 };

// Sums the partials in a fixed order and advances the CGLS scalars
// (Hestenes-Stiefel form):
//   start: gamma = gamma0 = |s0|^2
//   QQ:    alpha = gamma / |q|^2   (|q| = 0: breakdown, alpha = 0)
//   Gamma: gamma' = |s|^2, beta = gamma'/gamma, gamma = gamma', k += 1
//   RR:    |r|^2 into the history
// The stop flag is raised by a breakdown or when gamma falls to the threshold
// (tol^2 times the reference gamma, fixed at the start).
__global__ void __launch_bounds__(kRedThreads)
finalize(const double *__restrict__ partial, int nparts, double *__restrict__ sc, int mode,
         double *__restrict__ out, const double *__restrict__ stop)
{
    if (stopped(stop)) return;
    __shared__ double sh[kRedThreads / 64];
    double acc = 0.0;
    // fixed assignment of partials to threads and a fixed tree: deterministic
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) acc += partial[i];
    const double s = block_sum(acc, sh);
    if (threadIdx.x != 0) return;
    double *hist_g = sc + kCglsScalars;
    double *hist_r = hist_g + kCglsHistory;
    const int k = (int)sc[6];
    switch (mode) {
    case kFinStart:
        sc[0] = s; sc[4] = s; sc[6] = 0.0; sc[7] = 0.0;
        hist_g[0] = s;
        sc[kCglsThr] = sc[kCglsTol2] * (sc[kCglsRef] > 0.0 ? sc[kCglsRef] : s);
        sc[kCglsStop] = (sc[kCglsThr] > 0.0 && s <= sc[kCglsThr]) ? 1.0 : 0.0;
        break;
    case kFinQQ:
        sc[1] = s;
        if (s > 0.0 && sc[0] > 0.0) {
            sc[2] = sc[0] / s;
        } else {
            sc[2] = 0.0;
            sc[7] = 1.0;   // breakdown: A p = 0
            sc[kCglsStop] = 1.0;
        }
        break;
    case kFinGamma: {
        const double g = sc[0];
        sc[3] = g > 0.0 ? s / g : 0.0;
        sc[0] = s;
        sc[6] = k + 1;
        if (k + 1 < kCglsHistory) hist_g[k + 1] = s;
        if (sc[kCglsThr] > 0.0 && s <= sc[kCglsThr]) sc[kCglsStop] = 1.0;
        break;
    }
    case kFinRR:
        sc[5] = s;
        if (k < kCglsHistory) hist_r[k] = s;
        break;
    default:
        if (out) *out = s;
        break;
    }
}

// x += alpha p (volume), r -= alpha q (projections), with partial sums of |r|^2
__global__ void __launch_bounds__(kRedThreads)
update_xr(float *__restrict__ x, const float *__restrict__ p, int64_t nv, float *__restrict__ r,
          const float *__restrict__ q, int64_t np, const double *__restrict__ sc,
          double *__restrict__ partial, const double *__restrict__ stop)
{
    if (stopped(stop)) return;
    __shared__ double sh[kRedThreads / 64];
    const float alpha = (float)sc[2];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool vx = ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(p)) & 15) == 0;
    const bool vr = ((reinterpret_cast<uintptr_t>(r) | reinterpret_cast<uintptr_t>(q)) & 15) == 0;
    int64_t tx = 0, tr = 0;
    if (vx) {
        float4 *x4 = reinterpret_cast<float4 *>(x);
        const float4 *p4 = reinterpret_cast<const float4 *>(p);
        for (int64_t i = t0; i < nv / 4; i += stride) {
            float4 a = x4[i];
            const float4 b = p4[i];
            a.x = fmaf(alpha, b.x, a.x); a.y = fmaf(alpha, b.y, a.y);
            a.z = fmaf(alpha, b.z, a.z); a.w = fmaf(alpha, b.w, a.w);
            x4[i] = a;
        }
        tx = nv / 4 * 4;
    }
    for (int64_t i = tx + t0; i < nv; i += stride) x[i] = fmaf(alpha, p[i], x[i]);
    double acc = 0.0;
    if (vr) {
        float4 *r4 = reinterpret_cast<float4 *>(r);
        const float4 *q4 = reinterpret_cast<const float4 *>(q);
        for (int64_t i = t0; i < np / 4; i += stride) {
            float4 a = r4[i];
            const float4 b = q4[i];
            a.x = fmaf(-alpha, b.x, a.x); a.y = fmaf(-alpha, b.y, a.y);
            a.z = fmaf(-alpha, b.z, a.z); a.w = fmaf(-alpha, b.w, a.w);
            r4[i] = a;
            acc += (double)a.x * a.x + (double)a.y * a.y + (double)a.z * a.z + (double)a.w * a.w;
        }
        tr = np / 4 * 4;
    }
    for (int64_t i = tr + t0; i < np; i += stride) {
        const float a = fmaf(-alpha, q[i], r[i]);
        r[i] = a;
        acc += (double)a * a;
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// p = s + beta p   (beta from the device scalars; copy when init != 0)
__global__ void __launch_bounds__(kRedThreads)
update_p(float *__restrict__ p, const float *__restrict__ s, int64_t n, const double *__restrict__ sc,
         int init, const double *__restrict__ stop)
{
    if (stopped(stop)) return;
    const float beta = init ? 0.0f : (float)sc[3];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t tp = 0;
    if (((reinterpret_cast<uintptr_t>(p) | reinterpret_cast<uintptr_t>(s)) & 15) == 0) {
        float4 *p4 = reinterpret_cast<float4 *>(p);
        const float4 *s4 = reinterpret_cast<const float4 *>(s);
        for (int64_t i = t0; i < n / 4; i += stride) {
            const float4 a = s4[i];
            float4 b = init ? make_float4(0.f, 0.f, 0.f, 0.f) : p4[i];
            b.x = fmaf(beta, b.x, a.x); b.y = fmaf(beta, b.y, a.y);
            b.z = fmaf(beta, b.z, a.z); b.w = fmaf(beta, b.w, a.w);
            p4[i] = b;
        }
        tp = n / 4 * 4;
    }
    for (int64_t i = tp + t0; i < n; i += stride) p[i] = init ? s[i] : fmaf(beta, p[i], s[i]);
}

// r = b - q
__global__ void __launch_bounds__(kRedThreads)
residual(float *__restrict__ r, const float *__restrict__ b, const float *__restrict__ q, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        r[i] = b[i] - q[i];
}

// ---------------------------------------------------------------- OS-SART

__global__ void __launch_bounds__(kRedThreads)
fill(float *__restrict__ p, int64_t n, float val)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = val;
}

// For the count views of a subset (blocks of nm pixels, view_step apart):
// q = (b - q) / R, 0 where R = 0.
__global__ void __launch_bounds__(kRedThreads)
sart_residual(float *__restrict__ q, const float *__restrict__ b, const float *__restrict__ R, int64_t nm,
              int count, int64_t view_step)
{
    const int64_t n = nm * count;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int64_t j = (i / nm) * view_step + i % nm;
        const float r = R[j];
        q[j] = r != 0.0f ? (b[j] - q[j]) / r : 0.0f;
    }
}

// x += lam z / C where C != 0; then x = max(x, 0) if nonneg.
__global__ void __launch_bounds__(kRedThreads)
sart_update(float *__restrict__ x, const float *__restrict__ z, const float *__restrict__ C, int64_t n,
            float lam, int nonneg)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const float c = C[i];
        float v = x[i];
        if (c != 0.0f) v = fmaf(lam, z[i] / c, v);
        if (nonneg) v = fmaxf(v, 0.0f);
        x[i] = v;
    }
}

// ---------------------------------------------------------------- LSQR
// Scalars (FP64, device): see kLsqr* in cvp_internal.h.  Recurrences of
// Paige & Saunders (1982), Golub-Kahan bidiagonalisation with a QR update.

// y = x - sc[ci] * y with partial sums of |y|^2 (ci < 0: y = x)
__global__ void __launch_bounds__(kRedThreads)
axpby_norm(float *__restrict__ y, const float *__restrict__ x, int64_t n, const double *__restrict__ sc, int ci,
           double *__restrict__ partial)
{
    __shared__ double sh[kRedThreads / 64];
    const float c = ci >= 0 ? (float)sc[ci] : 0.0f;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const float v = ci >= 0 ? fmaf(-c, y[i], x[i]) : x[i];
        y[i] = v;
        acc += (double)v * v;
    }
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// y *= 1 / sc[ci] (left alone where sc[ci] = 0)
__global__ void __launch_bounds__(kRedThreads)
scale_by_inverse(float *__restrict__ y, int64_t n, const double *__restrict__ sc, int ci)
{
    const double d = sc[ci];
    if (!(d > 0.0)) return;
    const float inv = (float)(1.0 / d);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) y[i] *= inv;
}

// v /= alpha; then start: w = v;  iteration: x += (phi/rho) w, w = v - (theta/rho) w
__global__ void __launch_bounds__(kRedThreads)
lsqr_vxw(float *__restrict__ v, float *__restrict__ x, float *__restrict__ w, int64_t n,
         const double *__restrict__ sc, int init)
{
    const double a = sc[kLsqrAlpha];
    const float inv = a > 0.0 ? (float)(1.0 / a) : 1.0f;
    const float fx = (float)sc[kLsqrXStep], fw = (float)sc[kLsqrWStep];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const float vn = v[i] * inv;
        v[i] = vn;
        if (init) {
            w[i] = vn;
        } else {
            const float wi = w[i];
            x[i] = fmaf(fx, wi, x[i]);
            w[i] = fmaf(-fw, wi, vn);
        }
    }
}

__global__ void __launch_bounds__(kRedThreads)
lsqr_finalize(const double *__restrict__ partial, int nparts, double *__restrict__ sc, int mode)
{
    __shared__ double sh[kRedThreads / 64];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) acc += partial[i];
    const double t = block_sum(acc, sh);
    if (threadIdx.x != 0) return;
    const double nrm = sqrt(t);
    double *hr = sc + kLsqrScalars;
    double *har = hr + kCglsHistory;
    switch (mode) {
    case kLsqrFinBeta0:
        sc[kLsqrBeta] = nrm;
        sc[kLsqrPhibar] = nrm;
        sc[kLsqrK] = 0.0;
        sc[kLsqrBreak] = 0.0;
        sc[kLsqrXStep] = 0.0;
        sc[kLsqrWStep] = 0.0;
        break;
    case kLsqrFinAlpha0:
        sc[kLsqrAlpha] = nrm;
        sc[kLsqrRhobar] = nrm;
        sc[kLsqrArnorm0] = nrm * sc[kLsqrBeta];
        hr[0] = sc[kLsqrBeta];
        har[0] = nrm * sc[kLsqrBeta];
        break;
    case kLsqrFinBeta:
        sc[kLsqrBeta] = nrm;
        break;
    default: {   // kLsqrFinAlpha: alpha, then the QR step of the bidiagonal problem
        sc[kLsqrAlpha] = nrm;
        const double rhobar = sc[kLsqrRhobar], beta = sc[kLsqrBeta], phibar = sc[kLsqrPhibar];
        const double rho = hypot(rhobar, beta);
        const int k = (int)sc[kLsqrK] + 1;
        if (rho > 0.0) {
            const double c = rhobar / rho, sn = beta / rho;
            sc[kLsqrXStep] = c * phibar / rho;   // phi / rho
            sc[kLsqrWStep] = sn * nrm / rho;     // theta / rho
            sc[kLsqrRhobar] = -c * nrm;
            sc[kLsqrPhibar] = sn * phibar;
            if (k < kCglsHistory) {
                hr[k] = sn * phibar;
                har[k] = sn * phibar * nrm * fabs(c);
            }
        } else {   // the bidiagonalisation has ended: x stays
            sc[kLsqrXStep] = 0.0;
            sc[kLsqrWStep] = 0.0;
            sc[kLsqrBreak] = 1.0;
            if (k < kCglsHistory) {
                hr[k] = phibar;
                har[k] = 0.0;
            }
        }
        sc[kLsqrK] = k;
        break;
    }
    }
}

}  // namespace

hipError_t blas_dot(const float *a, const float *b, int64_t n, double *partials, double *sc,
                    int mode, double *out, hipStream_t s, const double *stop)
{
    hipLaunchKernelGGL(dot_partials, dim3(kRedBlocks), dim3(kRedThreads), 0, s, a, b, n, partials, stop);
    hipLaunchKernelGGL(finalize, dim3(1), dim3(kRedThreads), 0, s, partials, kRedBlocks, sc, mode, out, stop);
    return hipGetLastError();
}

hipError_t blas_update_xr(float *x, const float *p, int64_t nv, float *r, const float *q, int64_t np,
                          double *sc, double *partials, hipStream_t s, const double *stop)
{
    hipLaunchKernelGGL(update_xr, dim3(kRedBlocks), dim3(kRedThreads), 0, s, x, p, nv, r, q, np, sc,
                       partials, stop);
    hipLaunchKernelGGL(finalize, dim3(1), dim3(kRedThreads), 0, s, partials, kRedBlocks, sc,
                       (int)kFinRR, nullptr, stop);
    return hipGetLastError();
}

hipError_t blas_update_p(float *p, const float *sv, int64_t n, const double *sc, int init, hipStream_t s,
                         const double *stop)
{
    hipLaunchKernelGGL(update_p, dim3(kRedBlocks), dim3(kRedThreads), 0, s, p, sv, n, sc, init, stop);
    return hipGetLastError();
}

__global__ void set_tolerance(double *sc, double tol2, double ref)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        sc[kCglsTol2] = tol2;
        sc[kCglsRef] = ref;
    }
}

hipError_t blas_set_tolerance(double *sc, double tol2, double ref, hipStream_t s)
{
    hipLaunchKernelGGL(set_tolerance, dim3(1), dim3(64), 0, s, sc, tol2, ref);
    return hipGetLastError();
}

hipError_t blas_residual(float *r, const float *b, const float *q, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(residual, dim3(kRedBlocks), dim3(kRedThreads), 0, s, r, b, q, n);
    return hipGetLastError();
}

hipError_t blas_fill(float *p, int64_t n, float val, hipStream_t s)
{
    hipLaunchKernelGGL(fill, dim3(kRedBlocks), dim3(kRedThreads), 0, s, p, n, val);
    return hipGetLastError();
}

hipError_t sart_residual_views(float *q, const float *b, const float *R, int64_t nm, int count, int64_t view_step,
                               hipStream_t s)
{
    hipLaunchKernelGGL(sart_residual, dim3(kRedBlocks), dim3(kRedThreads), 0, s, q, b, R, nm, count, view_step);
    return hipGetLastError();
}

hipError_t sart_update_x(float *x, const float *z, const float *C, int64_t n, float lam, int nonneg, hipStream_t s)
{
    hipLaunchKernelGGL(sart_update, dim3(kRedBlocks), dim3(kRedThreads), 0, s, x, z, C, n, lam, nonneg);
    return hipGetLastError();
}

hipError_t lsqr_axpby_norm(float *y, const float *x, int64_t n, double *sc, int ci, int mode, hipStream_t s)
{
    double *part = sc + kLsqrScalars + 2 * kCglsHistory;
    hipLaunchKernelGGL(axpby_norm, dim3(kRedBlocks), dim3(kRedThreads), 0, s, y, x, n, sc, ci, part);
    hipLaunchKernelGGL(lsqr_finalize, dim3(1), dim3(kRedThreads), 0, s, part, kRedBlocks, sc, mode);
    return hipGetLastError();
}

hipError_t lsqr_norm(const float *a, int64_t n, double *sc, int mode, hipStream_t s)
{
    double *part = sc + kLsqrScalars + 2 * kCglsHistory;
    hipLaunchKernelGGL(dot_partials, dim3(kRedBlocks), dim3(kRedThreads), 0, s, a, a, n, part, nullptr);
    hipLaunchKernelGGL(lsqr_finalize, dim3(1), dim3(kRedThreads), 0, s, part, kRedBlocks, sc, mode);
    return hipGetLastError();
}

hipError_t lsqr_scale(float *y, int64_t n, const double *sc, int ci, hipStream_t s)
{
    hipLaunchKernelGGL(scale_by_inverse, dim3(kRedBlocks), dim3(kRedThreads), 0, s, y, n, sc, ci);
    return hipGetLastError();
}

hipError_t lsqr_update_vxw(float *v, float *x, float *w, int64_t n, const double *sc, int init, hipStream_t s)
{
    hipLaunchKernelGGL(lsqr_vxw, dim3(kRedBlocks), dim3(kRedThreads), 0, s, v, x, w, n, sc, init);
    return hipGetLastError();
}

}  // namespace cvp
