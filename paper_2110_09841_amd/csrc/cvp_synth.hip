// Input generation on the GPU for the learned warm start (not part of the
// projector): ellipsoid phantoms voxelised from host-drawn parameters, and
// Gaussian noise from a counter-based generator.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "cvp.h"

namespace {

// Sum of mu over the ellipsoids containing each voxel centre, FP64 with the
// same operation order as the host reference (contraction off), so the two
// agree bit for bit.  params: n x 16 doubles (centre, semi-axes, R, mu).
__global__ void ellipsoids_kernel(const double *__restrict__ params, int n, int n1, int n2, int n3,
                                  double a1, double a2, double a3, float *__restrict__ vol)
{
#pragma clang fp contract(off)
    const int64_t nv = (int64_t)n1 * n2 * n3;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(v % n1), j = (int)((v / n1) % n2), k = (int)(v / ((int64_t)n1 * n2));
        const double x = (i - (n1 - 1) / 2.0) * a1, y = (j - (n2 - 1) / 2.0) * a2, z = (k - (n3 - 1) / 2.0) * a3;
        double acc = 0.0;
        for (int e = 0; e < n; ++e) {
            const double *P = params + 16 * e;
            const double X = x - P[0], Y = y - P[1], Z = z - P[2];
            const double px = P[6] * X + P[9] * Y + P[12] * Z;
            const double py = P[7] * X + P[10] * Y + P[13] * Z;
            const double pz = P[8] * X + P[11] * Y + P[14] * Z;
            const double qx = px / P[3], qy = py / P[4], qz = pz / P[5];
            if (qx * qx + qy * qy + qz * qz <= 1.0) acc += P[15];
        }
        vol[v] = (float)acc;
    }
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011).
__device__ __forceinline__ void philox(uint32_t c[4], uint32_t k0, uint32_t k1)
{
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// out[i] += sigma * N(0,1): counter (i/4, 0, 0, 0), key = seed; Box-Muller on
// pairs of the four 32-bit outputs.
__global__ void gaussian_kernel(float *__restrict__ out, int64_t n, float sigma, uint64_t seed)
{
    const int64_t nq = (n + 3) / 4;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nq; q += (int64_t)gridDim.x * blockDim.x) {
        uint32_t c[4] = {(uint32_t)q, (uint32_t)(q >> 32), 0u, 0u};
        philox(c, (uint32_t)seed, (uint32_t)(seed >> 32));
        float z[4];
        for (int h = 0; h < 2; ++h) {
            const float u1 = ((float)c[2 * h] + 0.5f) * 2.3283064365386963e-10f;   // (0, 1)
            const float u2 = ((float)c[2 * h + 1] + 0.5f) * 2.3283064365386963e-10f;
            const float r = sqrtf(-2.0f * logf(u1));
            z[2 * h] = r * cosf(6.283185307179586f * u2);
            z[2 * h + 1] = r * sinf(6.283185307179586f * u2);
        }
        for (int e = 0; e < 4; ++e) {
            const int64_t i = 4 * q + e;
            if (i < n) out[i] += sigma * z[e];
        }
    }
}

}  // namespace

extern "C" {

cvp_status cvp_synth_ellipsoids(const double *d_params, int32_t n, const int32_t dims[3],
                                const double voxel_mm[3], float *d_vol, void *stream)
{
    if (!d_params || n < 0 || !dims || !voxel_mm || !d_vol) return CVP_E_INVALID;
    if (dims[0] <= 0 || dims[1] <= 0 || dims[2] <= 0) return CVP_E_INVALID;
    const int64_t nv = (int64_t)dims[0] * dims[1] * dims[2];
    const int grid = (int)((nv + 255) / 256 < 8192 ? (nv + 255) / 256 : 8192);
    hipLaunchKernelGGL(ellipsoids_kernel, dim3(grid), dim3(256), 0, (hipStream_t)stream, d_params, n, dims[0],
                       dims[1], dims[2], voxel_mm[0], voxel_mm[1], voxel_mm[2], d_vol);
    return hipGetLastError() == hipSuccess ? CVP_OK : CVP_E_DEVICE;
}

cvp_status cvp_synth_add_gaussian(float *d_out, int64_t n, float sigma, uint64_t seed, void *stream)
{
    if (!d_out || n < 0) return CVP_E_INVALID;
    const int64_t nq = (n + 3) / 4;
    const int grid = (int)((nq + 255) / 256 < 8192 ? (nq + 255) / 256 : 8192);
    hipLaunchKernelGGL(gaussian_kernel, dim3(grid), dim3(256), 0, (hipStream_t)stream, d_out, n, sigma, seed);
    return hipGetLastError() == hipSuccess ? CVP_OK : CVP_E_DEVICE;
}

}  // extern "C"
