// Kernels of the learned CGLS warm start: a small 3D U-Net with 3x3x3
// convolutions, BF16 activations and weights, FP32 accumulation.
//
// Layout: channels last, [D][H][W][C] BF16, with an explicit channel stride
// (so a tensor can be a channel slice of a wider one: concatenation costs
// nothing) and channel counts that are multiples of 8.
//
// conv3d (forward and backward-data) is an implicit GEMM on the MFMA unit:
//   out[v][co] = sum_k A[v][k] B[k][co],  k = tap * Cin + ci,  27 taps,
// with v_mfma_f32_16x16x32_bf16.  Lane l of a wave holds, for the 16x32 A
// tile, row l%16 and the 8 consecutive k of group l/16 -- 8 consecutive input
// channels of one tap, i.e. one 16-byte load in channels-last layout; the B
// tile likewise holds 8 consecutive input channels of one output channel
// (weights stored [tap][co][ci]).  The 16x16 FP32 result has row 4*(l/16)+e,
// column l%16 in element e of lane l.
// conv3d backward-weight reduces over voxels: D[co][ci] = sum_v dY[v][co] X[v+off][ci],
// with dY and the shifted X rows staged transposed in LDS so that the 8
// consecutive voxels of a lane are one 16-byte LDS read.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

namespace cvpnn {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

struct Act {             // a channels-last BF16 tensor (or channel slice)
    __bf16 *p;
    int D, H, W;
    int C;               // channels used
    int stride;          // channels between consecutive voxels (>= C)
};

__device__ __forceinline__ bf16x8 zero8()
{
    bf16x8 z;
#pragma unroll
    for (int e = 0; e < 8; ++e) z[e] = (__bf16)0.0f;
    return z;
}

// ------------------------------------------------------------------ conv3d

// One wave computes 64 consecutive voxels of one (d, h) row (4 row tiles of
// 16) for all output channels (CO/16 column tiles).  Weights wt: [27][Co][Ci].
// flip = 1 mirrors the taps (used by backward-data with the transposed
// weights).  relu = 1 applies max(., 0) before the BF16 store.
template <int CO>
__global__ void __launch_bounds__(256)
conv3d_kernel(const Act in, const __bf16 *__restrict__ wt, const float *__restrict__ bias,
              Act out, int relu, int flip)
{
    constexpr int NT = CO / 16;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int segs = (in.W + 63) / 64;
    const int row = blockIdx.x * 4 + wave;           // (d, h, segment)
    if (row >= in.D * in.H * segs) return;
    const int seg = row % segs;
    const int dh = row / segs;
    const int d = dh / in.H, h = dh % in.H;
    const int w0 = seg * 64;
    const int Ci = in.C;
    const int K = 27 * Ci;
    const int ksteps = (K + 31) / 32;

    f32x4 acc[4][NT];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int n = 0; n < NT; ++n) acc[r][n] = f32x4{0.f, 0.f, 0.f, 0.f};

    const int i16 = lane & 15;
    const int kg = lane >> 4;        // which group of 8 k within the 32
    for (int ks = 0; ks < ksteps; ++ks) {
        const int k = ks * 32 + kg * 8;
        const int tap = k / Ci;
        const int ci = k - tap * Ci;
        const bool tv = tap < 27;
        const int tp = flip ? 26 - tap : tap;
        const int dz = tp / 9 - 1, dy = (tp / 3) % 3 - 1, dx = tp % 3 - 1;
        const int z = d + dz, y = h + dy;
        const bool zy = tv && z >= 0 && z < in.D && y >= 0 && y < in.H;
        bf16x8 a[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int x = w0 + r * 16 + i16 + dx;
            if (zy && x >= 0 && x < in.W)
                a[r] = *reinterpret_cast<const bf16x8 *>(in.p + (((size_t)z * in.H + y) * in.W + x) * in.stride + ci);
            else
                a[r] = zero8();
        }
#pragma unroll
        for (int n = 0; n < NT; ++n) {
            const int co = n * 16 + i16;
            bf16x8 b = tv ? *reinterpret_cast<const bf16x8 *>(wt + ((size_t)tap * CO + co) * Ci + ci) : zero8();
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[r][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[r], b, acc[r][n], 0, 0, 0);
        }
    }
    // epilogue: lane holds rows 4*(l/16)+e, column l%16 of each tile
#pragma unroll
    for (int n = 0; n < NT; ++n) {
        const int co = n * 16 + i16;
        const float bv = bias ? bias[co] : 0.0f;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int x = w0 + r * 16 + (lane >> 4) * 4 + e;
                if (x < out.W) {
                    float v = acc[r][n][e] + bv;
                    if (relu) v = fmaxf(v, 0.0f);
                    out.p[(((size_t)d * out.H + h) * out.W + x) * out.stride + co] = (__bf16)v;
                }
            }
        }
    }
}

// The same convolution with the input channel count CI a compile-time power
// of two (16, 32 or 64), for volumes whose element count fits 32 bits: a
// lane's tap and channel follow from shifts, the tap's offsets from
// divisions by constants, and the addresses from 32-bit voxel indices.  The
// arithmetic (k order, MFMA sequence, epilogue) is that of conv3d_kernel, so
// the results are the same bits.
template <int CO, int CI>
__global__ void __launch_bounds__(256)
conv3d_kernel_c(const Act in, const __bf16 *__restrict__ wt, const float *__restrict__ bias, Act out, int relu,
                int flip)
{
    constexpr int NT = CO / 16;
    constexpr int KSTEPS = (27 * CI + 31) / 32;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int segs = (in.W + 63) / 64;
    const int row = blockIdx.x * 4 + wave;           // (d, h, segment)
    if (row >= in.D * in.H * segs) return;
    const int seg = row % segs;
    const int dh = row / segs;
    const int d = dh / in.H, h = dh % in.H;
    const int w0 = seg * 64;

    f32x4 acc[4][NT];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int n = 0; n < NT; ++n) acc[r][n] = f32x4{0.f, 0.f, 0.f, 0.f};

    const int i16 = lane & 15;
    const int kg = lane >> 4;        // which group of 8 k within the 32
#pragma unroll 2
    for (int ks = 0; ks < KSTEPS; ++ks) {
        const int k = ks * 32 + kg * 8;
        const int tap = k / CI;
        const int ci = k % CI;
        const bool tv = tap < 27;
        const int tp = flip ? 26 - tap : tap;
        const int dz = tp / 9 - 1, dy = (tp / 3) % 3 - 1, dx = tp % 3 - 1;
        const int z = d + dz, y = h + dy;
        const bool zy = tv && (unsigned)z < (unsigned)in.D && (unsigned)y < (unsigned)in.H;
        const int base = (z * in.H + y) * in.W + w0 + i16 + dx;   // voxel index of row tile 0
        bf16x8 a[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int x = w0 + r * 16 + i16 + dx;
            if (zy && (unsigned)x < (unsigned)in.W)
                a[r] = *reinterpret_cast<const bf16x8 *>(in.p + (base + r * 16) * in.stride + ci);
            else
                a[r] = zero8();
        }
#pragma unroll
        for (int n = 0; n < NT; ++n) {
            const int co = n * 16 + i16;
            bf16x8 b = tv ? *reinterpret_cast<const bf16x8 *>(wt + (tap * CO + co) * CI + ci) : zero8();
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[r][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[r], b, acc[r][n], 0, 0, 0);
        }
    }
#pragma unroll
    for (int n = 0; n < NT; ++n) {
        const int co = n * 16 + i16;
        const float bv = bias ? bias[co] : 0.0f;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int x = w0 + r * 16 + (lane >> 4) * 4 + e;
                if (x < out.W) {
                    float v = acc[r][n][e] + bv;
                    if (relu) v = fmaxf(v, 0.0f);
                    out.p[((d * out.H + h) * out.W + x) * out.stride + co] = (__bf16)v;
                }
            }
        }
    }
}

// The same convolution with the workgroup's input tile staged in LDS: a
// workgroup computes 16 RX voxels (RX = 4 or 2 row tiles per wave) of 4
// consecutive rows h0..h0+3 of slice d (one row per wave) and first copies the
// (16 RX + 2) x 6 x 3 input voxels those outputs read (zeros outside the
// volume) into LDS, so each of the 27
// taps' A fragments is an LDS read instead of a gather from global memory
// (every input voxel was fetched 27 times through L1).  The k order, MFMA
// sequence and epilogue are those of conv3d_kernel: the results are the same
// bits.  RX = 4 with 16 or 32 input channels (38 or 76 KB of LDS), RX = 2
// with 64 (78 KB).
constexpr int kTileY = 6, kTileZ = 3;

template <int CI, int RX>
constexpr int conv_tile_bytes() { return kTileZ * kTileY * (RX * 16 + 2) * CI * 2; }

// LDS holds 4 (16 input channels) or 2 (32) workgroups per CU: the register
// budget of that occupancy lets the scheduler keep more fragments in flight.
template <int CO, int CI, int RX>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(conv_tile_bytes<CI, RX>() <= 40960 ? 4 : 2)))
conv3d_lds_kernel(const Act in, const __bf16 *__restrict__ wt, const float *__restrict__ bias, Act out, int relu,
                  int flip)
{
    constexpr int NT = CO / 16;
    constexpr int KSTEPS = (27 * CI + 31) / 32;
    constexpr int C8 = CI / 8;                       // 16-byte chunks per voxel
    extern __shared__ __align__(16) unsigned char tile[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int kTileX = RX * 16 + 2;
    const int segs = (in.W + RX * 16 - 1) / (RX * 16), quads = (in.H + 3) / 4;
    int blk = blockIdx.x;
    const int seg = blk % segs;
    blk /= segs;
    const int h0 = (blk % quads) * 4;
    const int d = blk / quads;
    const int w0 = seg * RX * 16;

    // stage the input tile, voxel v = (zz, yy, xx) = (d - 1 + zz, h0 - 1 + yy,
    // w0 - 1 + xx), as [8-channel chunk][voxel][16 bytes]: the 16 lanes of a
    // fragment read consecutive 16-byte slots (no LDS bank conflicts)
    constexpr int NV = kTileZ * kTileY * kTileX;
    constexpr int NCH = NV * C8;
    for (int idx = threadIdx.x; idx < NCH; idx += 256) {
        const int c8 = idx / NV, v = idx % NV;
        const int xx = v % kTileX, t = v / kTileX;
        const int yy = t % kTileY, zz = t / kTileY;
        const int x = w0 - 1 + xx, y = h0 - 1 + yy, z = d - 1 + zz;
        bf16x8 val = zero8();
        if ((unsigned)x < (unsigned)in.W && (unsigned)y < (unsigned)in.H && (unsigned)z < (unsigned)in.D)
            val = *reinterpret_cast<const bf16x8 *>(in.p + ((z * in.H + y) * in.W + x) * in.stride + c8 * 8);
        *reinterpret_cast<bf16x8 *>(tile + idx * 16) = val;
    }
    __syncthreads();
    const int h = h0 + wave;
    if (h >= in.H) return;                           // no barrier follows

    f32x4 acc[RX][NT];
#pragma unroll
    for (int r = 0; r < RX; ++r)
#pragma unroll
        for (int n = 0; n < NT; ++n) acc[r][n] = f32x4{0.f, 0.f, 0.f, 0.f};

    const int i16 = lane & 15;
    const int kg = lane >> 4;        // which group of 8 k within the 32
    // fragments of k step ks: A from the tile, B (weights) from global memory
    auto load = [&](int ks, bf16x8 a[RX], bf16x8 b[NT]) {
        const int k = ks * 32 + kg * 8;
        const int tap = k / CI;
        const int ci = k % CI;
        const bool tv = tap < 27;
        const int tp = flip ? 26 - tap : tap;
        const int dz = tp / 9 - 1, dy = (tp / 3) % 3 - 1, dx = tp % 3 - 1;
        // tile voxel of row tile 0: (dz + 1, wave + dy + 1, i16 + dx + 1)
        const unsigned char *src =
            tile + ((ci / 8) * NV + ((dz + 1) * kTileY + wave + dy + 1) * kTileX + i16 + dx + 1) * 16;
#pragma unroll
        for (int r = 0; r < RX; ++r) a[r] = tv ? *reinterpret_cast<const bf16x8 *>(src + r * 16 * 16) : zero8();
#pragma unroll
        for (int n = 0; n < NT; ++n)
            b[n] = tv ? *reinterpret_cast<const bf16x8 *>(wt + (tap * CO + n * 16 + i16) * CI + ci) : zero8();
    };
    // the k loop unrolled, with the next step's fragments loaded before this
    // step's MFMAs (two register sets)
    bf16x8 fa[2][RX], fb[2][NT];
    load(0, fa[0], fb[0]);
#pragma unroll
    for (int ks = 0; ks < KSTEPS; ++ks) {
        const int c = ks & 1;
        if (ks + 1 < KSTEPS) load(ks + 1, fa[c ^ 1], fb[c ^ 1]);
#pragma unroll
        for (int n = 0; n < NT; ++n)
#pragma unroll
            for (int r = 0; r < RX; ++r)
                acc[r][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[c][r], fb[c][n], acc[r][n], 0, 0, 0);
    }
#pragma unroll
    for (int n = 0; n < NT; ++n) {
        const int co = n * 16 + i16;
        const float bv = bias ? bias[co] : 0.0f;
#pragma unroll
        for (int r = 0; r < RX; ++r) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int x = w0 + r * 16 + (lane >> 4) * 4 + e;
                if (x < out.W) {
                    float v = acc[r][n][e] + bv;
                    if (relu) v = fmaxf(v, 0.0f);
                    out.p[((d * out.H + h) * out.W + x) * out.stride + co] = (__bf16)v;
                }
            }
        }
    }
}

// Backward-weight partials: for the taps (dz, dy) = tap9 and all three dx,
// and a chunk of `rows` (d, h) rows, part[chunk][tap][co][ci] =
// sum over the chunk's voxels of dY[v][co] * X[v + off][ci].  Per 64-voxel
// segment, dY and the three dx-shifted X rows are staged transposed in LDS
// as [channel][voxel pair]: a thread loads 8 channels of two neighbouring
// voxels (two 16-byte loads) and writes 8 words each holding the channel's
// two BF16 values, so the writes of a wave are consecutive words.  A lane's
// MFMA fragment (8 consecutive voxels of one channel) is then one 16-byte
// LDS read; the row pitch of 36 words keeps those reads conflict free.
// Wave w owns the 16x16 (co, ci) tiles w, w + 4, ...
template <int CO, int CI>
__global__ void __launch_bounds__(256)
conv3d_wgrad_kernel(const Act x, const Act dy, int rows_per_chunk, float *__restrict__ part)
{
    constexpr int MT = CO / 16, NT = CI / 16;
    constexpr int TILES = MT * NT;                 // 16x16 tiles per tap
    constexpr int PER_WAVE = (TILES + 3) / 4;
    constexpr int PITCH = 36;                      // words per channel row (32 voxel pairs + pad)
    __shared__ __align__(16) unsigned sdy[CO * PITCH];
    __shared__ __align__(16) unsigned sx[3 * CI * PITCH];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int tap9 = blockIdx.y;                   // (dz, dy) in 0..8
    const int dz = tap9 / 3 - 1, dyo = tap9 % 3 - 1;
    const int chunk = blockIdx.x;
    const int nrows = x.D * x.H;
    const int r0 = chunk * rows_per_chunk;
    const int r1 = min(r0 + rows_per_chunk, nrows);
    const int segs = (x.W + 63) / 64;

    f32x4 acc[3][PER_WAVE];
#pragma unroll
    for (int t = 0; t < 3; ++t)
#pragma unroll
        for (int q = 0; q < PER_WAVE; ++q) acc[t][q] = f32x4{0.f, 0.f, 0.f, 0.f};

    // 8 channels of voxel w of a row (zero outside [0, W) or when !ok)
    auto load8 = [](const Act &a, size_t rowbase, int w, int c0, bool ok) {
        if (ok && w >= 0 && w < a.W)
            return *reinterpret_cast<const bf16x8 *>(a.p + (rowbase + w) * a.stride + c0);
        return zero8();
    };
    auto pack = [](__bf16 lo, __bf16 hi) {
        return (unsigned)__builtin_bit_cast(unsigned short, lo) | ((unsigned)__builtin_bit_cast(unsigned short, hi) << 16);
    };

    for (int rr = r0; rr < r1; ++rr) {
        const int d = rr / x.H, h = rr % x.H;
        const int z = d + dz, y = h + dyo;
        const bool zy = z >= 0 && z < x.D && y >= 0 && y < x.H;
        const size_t dyrow = ((size_t)d * dy.H + h) * dy.W;
        const size_t xrow = ((size_t)z * x.H + y) * x.W;
        for (int seg = 0; seg < segs; ++seg) {
            const int w0 = seg * 64;
            __syncthreads();
            // dY: tasks (pair m, channel group g)
            for (int task = threadIdx.x; task < 32 * (CO / 8); task += 256) {
                const int m = task & 31, g = task >> 5;
                const int wa = w0 + 2 * m;
                const bf16x8 a = load8(dy, dyrow, wa, 8 * g, true);
                const bf16x8 b = load8(dy, dyrow, wa + 1, 8 * g, true);
#pragma unroll
                for (int e = 0; e < 8; ++e) sdy[(8 * g + e) * PITCH + m] = pack(a[e], b[e]);
            }
            // X, three dx shifts: tasks (pair m, channel group g, shift t)
            for (int task = threadIdx.x; task < 3 * 32 * (CI / 8); task += 256) {
                const int m = task & 31, g = (task >> 5) % (CI / 8), t = task / (32 * (CI / 8));
                const int va = 2 * m, wa = w0 + va + t - 1;
                const bf16x8 a = load8(x, xrow, wa, 8 * g, zy && w0 + va < x.W);
                const bf16x8 b = load8(x, xrow, wa + 1, 8 * g, zy && w0 + va + 1 < x.W);
#pragma unroll
                for (int e = 0; e < 8; ++e) sx[(t * CI + 8 * g + e) * PITCH + m] = pack(a[e], b[e]);
            }
            __syncthreads();
            // K = 64 voxels = 2 MFMA steps of 32; lane reads voxels v0 .. v0+7
#pragma unroll
            for (int ks = 0; ks < 2; ++ks) {
                const int p0 = ks * 16 + (lane >> 4) * 4;          // first voxel pair
#pragma unroll
                for (int q = 0; q < PER_WAVE; ++q) {
                    const int tile = wave + 4 * q;
                    if (tile < TILES) {
                        const int mt = tile / NT, nt = tile % NT;
                        const bf16x8 a = *reinterpret_cast<const bf16x8 *>(&sdy[(mt * 16 + (lane & 15)) * PITCH + p0]);
#pragma unroll
                        for (int t = 0; t < 3; ++t) {
                            const bf16x8 b =
                                *reinterpret_cast<const bf16x8 *>(&sx[(t * CI + nt * 16 + (lane & 15)) * PITCH + p0]);
                            acc[t][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[t][q], 0, 0, 0);
                        }
                    }
                }
            }
        }
    }
    // part layout: [chunk][27][CO][CI]; tap = tap9 * 3 + (dx + 1)
#pragma unroll
    for (int q = 0; q < PER_WAVE; ++q) {
        const int tile = wave + 4 * q;
        if (tile >= TILES) continue;
        const int mt = tile / NT, nt = tile % NT;
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            float *dst = part + (((size_t)chunk * 27 + tap9 * 3 + t) * CO) * CI;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int co = mt * 16 + (lane >> 4) * 4 + e;
                const int ci = nt * 16 + (lane & 15);
                dst[co * CI + ci] = acc[t][q][e];
            }
        }
    }
}

// out[i] = sum over chunks of part[chunk][i], i < n.  A block takes 64
// consecutive i; wave w sums the chunks c = w, w + 4, ... in order and the
// four wave sums are added in a fixed order (deterministic).
__global__ void reduce_chunks(const float *__restrict__ part, int chunks, int64_t n, float *__restrict__ out)
{
    __shared__ float red[4][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int64_t base = (int64_t)blockIdx.x * 64; base < n; base += (int64_t)gridDim.x * 64) {
        const int64_t i = base + lane;
        float s = 0.0f;
        if (i < n)
            for (int c = wave; c < chunks; c += 4) s += part[(size_t)c * n + i];
        red[wave][lane] = s;
        __syncthreads();
        if (wave == 0 && i < n) out[i] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
        __syncthreads();
    }
}

// Per-channel sums over voxels (bias gradient), partials per block row chunk.
// Thread t takes channel group t % (C/8) of every (256/(C/8))-th voxel with
// 16-byte loads; the block then adds the per-thread sums of each channel in
// a fixed order.
__global__ void channel_sum_partials(const Act a, int rows_per_chunk, float *__restrict__ part)
{
    __shared__ float red[256 * 8];
    const int chunk = blockIdx.x;
    const int nvox = a.D * a.H * a.W;
    const int v0 = chunk * rows_per_chunk * a.W;
    const int v1 = min(v0 + rows_per_chunk * a.W, nvox);
    const int groups = a.C / 8;
    const int g = threadIdx.x % groups, lanes = 256 / groups;
    const int vt = threadIdx.x / groups;
    float s[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) s[e] = 0.0f;
    if (vt < lanes) {
        for (int v = v0 + vt; v < v1; v += lanes) {
            const bf16x8 q = *reinterpret_cast<const bf16x8 *>(a.p + (size_t)v * a.stride + 8 * g);
#pragma unroll
            for (int e = 0; e < 8; ++e) s[e] += (float)q[e];
        }
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) red[threadIdx.x * 8 + e] = s[e];
    __syncthreads();
    for (int c = threadIdx.x; c < a.C; c += 256) {
        const int gg = c / 8, e = c % 8;
        float t = 0.0f;
        for (int k = 0; k < lanes; ++k) t += red[(k * groups + gg) * 8 + e];
        part[(size_t)chunk * a.C + c] = t;
    }
}

// Elementwise kernels: one thread per 8-channel chunk of a voxel (16-byte
// loads and stores), index I = int when the chunk count fits 31 bits.  Each
// value is computed as in a per-channel loop, in the same order.
template <typename I>
__device__ __forceinline__ void chunk_coords(I i, int C8, int W, int H, int &c, int &x, int &y, int &z)
{
    c = (int)(i % C8) * 8;
    I v = i / C8;
    x = (int)(v % W);
    v /= W;
    y = (int)(v % H);
    z = (int)(v / H);
}

__device__ __forceinline__ size_t voxel_at(const Act &t, int z, int y, int x)
{
    return (((size_t)z * t.H + y) * t.W + x) * t.stride;
}

// dY *= (Y > 0) in place (ReLU backward; Y is the post-ReLU output)
template <typename I>
__global__ void relu_mask(Act dy, const Act y)
{
    const int C8 = dy.C / 8;
    const I n = (I)dy.D * dy.H * dy.W * C8;
    for (I i = (I)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (I)gridDim.x * blockDim.x) {
        const I v = i / C8;
        const int c = (int)(i % C8) * 8;
        bf16x8 g = *reinterpret_cast<const bf16x8 *>(dy.p + (size_t)v * dy.stride + c);
        const bf16x8 q = *reinterpret_cast<const bf16x8 *>(y.p + (size_t)v * y.stride + c);
#pragma unroll
        for (int e = 0; e < 8; ++e)
            if (!((float)q[e] > 0.0f)) g[e] = (__bf16)0.0f;
        *reinterpret_cast<bf16x8 *>(dy.p + (size_t)v * dy.stride + c) = g;
    }
}

// 2x2x2 average pooling: out (D/2,H/2,W/2) from in
template <typename I>
__global__ void avgpool2(const Act in, Act out)
{
    const int C8 = out.C / 8;
    const I n = (I)out.D * out.H * out.W * C8;
    for (I i = (I)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (I)gridDim.x * blockDim.x) {
        int c, x, y, z;
        chunk_coords<I>(i, C8, out.W, out.H, c, x, y, z);
        float s[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) s[e] = 0.0f;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const bf16x8 t = *reinterpret_cast<const bf16x8 *>(
                in.p + voxel_at(in, 2 * z + (q >> 2), 2 * y + ((q >> 1) & 1), 2 * x + (q & 1)) + c);
#pragma unroll
            for (int e = 0; e < 8; ++e) s[e] += (float)t[e];
        }
        bf16x8 o;
#pragma unroll
        for (int e = 0; e < 8; ++e) o[e] = (__bf16)(0.125f * s[e]);
        *reinterpret_cast<bf16x8 *>(out.p + voxel_at(out, z, y, x) + c) = o;
    }
}

// backward of avgpool2: din = dout(parent) / 8
template <typename I>
__global__ void avgpool2_bwd(const Act dout, Act din)
{
    const int C8 = din.C / 8;
    const I n = (I)din.D * din.H * din.W * C8;
    for (I i = (I)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (I)gridDim.x * blockDim.x) {
        int c, x, y, z;
        chunk_coords<I>(i, C8, din.W, din.H, c, x, y, z);
        const bf16x8 g = *reinterpret_cast<const bf16x8 *>(dout.p + voxel_at(dout, z / 2, y / 2, x / 2) + c);
        bf16x8 o;
#pragma unroll
        for (int e = 0; e < 8; ++e) o[e] = (__bf16)(0.125f * (float)g[e]);
        *reinterpret_cast<bf16x8 *>(din.p + voxel_at(din, z, y, x) + c) = o;
    }
}

// nearest 2x upsampling: out (2D,2H,2W) from in
template <typename I>
__global__ void upsample2(const Act in, Act out)
{
    const int C8 = out.C / 8;
    const I n = (I)out.D * out.H * out.W * C8;
    for (I i = (I)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (I)gridDim.x * blockDim.x) {
        int c, x, y, z;
        chunk_coords<I>(i, C8, out.W, out.H, c, x, y, z);
        *reinterpret_cast<bf16x8 *>(out.p + voxel_at(out, z, y, x) + c) =
            *reinterpret_cast<const bf16x8 *>(in.p + voxel_at(in, z / 2, y / 2, x / 2) + c);
    }
}

// backward of upsample2: din = sum of the 8 children of dout
template <typename I>
__global__ void upsample2_bwd(const Act dout, Act din)
{
    const int C8 = din.C / 8;
    const I n = (I)din.D * din.H * din.W * C8;
    for (I i = (I)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (I)gridDim.x * blockDim.x) {
        int c, x, y, z;
        chunk_coords<I>(i, C8, din.W, din.H, c, x, y, z);
        float s[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) s[e] = 0.0f;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const bf16x8 t = *reinterpret_cast<const bf16x8 *>(
                dout.p + voxel_at(dout, 2 * z + (q >> 2), 2 * y + ((q >> 1) & 1), 2 * x + (q & 1)) + c);
#pragma unroll
            for (int e = 0; e < 8; ++e) s[e] += (float)t[e];
        }
        bf16x8 o;
#pragma unroll
        for (int e = 0; e < 8; ++e) o[e] = (__bf16)s[e];
        *reinterpret_cast<bf16x8 *>(din.p + voxel_at(din, z, y, x) + c) = o;
    }
}

// out = a + b (BF16 tensors of the same shape; slices allowed)
template <typename I>
__global__ void add_kernel(const Act a, const Act b, Act out)
{
    const int C8 = out.C / 8;
    const I n = (I)out.D * out.H * out.W * C8;
    for (I i = (I)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (I)gridDim.x * blockDim.x) {
        const I v = i / C8;
        const int c = (int)(i % C8) * 8;
        const bf16x8 p = *reinterpret_cast<const bf16x8 *>(a.p + (size_t)v * a.stride + c);
        const bf16x8 q = *reinterpret_cast<const bf16x8 *>(b.p + (size_t)v * b.stride + c);
        bf16x8 o;
#pragma unroll
        for (int e = 0; e < 8; ++e) o[e] = (__bf16)((float)p[e] + (float)q[e]);
        *reinterpret_cast<bf16x8 *>(out.p + (size_t)v * out.stride + c) = o;
    }
}

// Pack two FP32 volumes into channels 0 and 1 of a 16-channel BF16 tensor
// (channels 2..15 zero), scaled by `scale`.
__global__ void pack_input(const float *__restrict__ x1, const float *__restrict__ x2, int64_t nvox,
                           float scale, Act out)
{
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nvox; v += (int64_t)gridDim.x * blockDim.x) {
        __bf16 *o = out.p + v * out.stride;
        bf16x8 a = zero8(), b = zero8();
        a[0] = (__bf16)(scale * x1[v]);
        a[1] = (__bf16)(scale * x2[v]);
        *reinterpret_cast<bf16x8 *>(o) = a;
        *reinterpret_cast<bf16x8 *>(o + 8) = b;
    }
}

// Output head (1x1x1 convolution 16 -> 1, in FP32) with the residual on x2:
//   x0 = x2 + (sum_c w[c] h[v][c] + b) / scale
__global__ void head_fwd(const Act h, const float *__restrict__ w, const float *__restrict__ b,
                         const float *__restrict__ x2, float inv_scale, float *__restrict__ x0)
{
    const int64_t n = (int64_t)h.D * h.H * h.W;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        float s = b[0];
        for (int c8 = 0; c8 < h.C; c8 += 8) {
            const bf16x8 q = *reinterpret_cast<const bf16x8 *>(h.p + v * h.stride + c8);
#pragma unroll
            for (int e = 0; e < 8; ++e) s = fmaf(w[c8 + e], (float)q[e], s);
        }
        x0[v] = x2[v] + s * inv_scale;
    }
}

// Head backward: dh[v][c] = w[c] g[v] / scale (BF16), partial sums for dw, db
__global__ void head_bwd(const Act h, const float *__restrict__ w, const float *__restrict__ g,
                         float inv_scale, Act dh, int64_t per_block, float *__restrict__ part)
{
    __shared__ float sh[17][256];
    const int64_t n = (int64_t)h.D * h.H * h.W;
    const int64_t v0 = (int64_t)blockIdx.x * per_block;
    const int64_t v1 = v0 + per_block < n ? v0 + per_block : n;
    float acc[17];
    for (int c = 0; c < 17; ++c) acc[c] = 0.0f;
    for (int64_t v = v0 + threadIdx.x; v < v1; v += blockDim.x) {
        const float gv = g[v] * inv_scale;
#pragma unroll
        for (int c8 = 0; c8 < 16; c8 += 8) {
            if (c8 >= h.C) break;
            const bf16x8 q = *reinterpret_cast<const bf16x8 *>(h.p + v * h.stride + c8);
            bf16x8 o;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                acc[c8 + e] = fmaf((float)q[e], gv, acc[c8 + e]);
                o[e] = (__bf16)(w[c8 + e] * gv);
            }
            *reinterpret_cast<bf16x8 *>(dh.p + v * dh.stride + c8) = o;
        }
        acc[16] += gv;
    }
    for (int c = 0; c < 17; ++c) sh[c][threadIdx.x] = acc[c];
    __syncthreads();
    if (threadIdx.x < 17) {
        float s = 0.0f;
        for (int t = 0; t < (int)blockDim.x; ++t) s += sh[threadIdx.x][t];
        part[(size_t)blockIdx.x * 17 + threadIdx.x] = s;
    }
}

// Weights [27][Co][Ci] -> [27][Ci][Co] (backward-data uses the mirrored taps)
__global__ void transpose_weights(const __bf16 *__restrict__ w, __bf16 *__restrict__ wt, int co, int ci)
{
    const int n = 27 * co * ci;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int t = i / (co * ci), r = i % (co * ci);
        const int o = r / ci, c = r % ci;
        wt[((size_t)t * ci + c) * co + o] = w[i];
    }
}

// MSE: grad = 2 (a - b) / n, partial sums of (a - b)^2 (FP64)
__global__ void mse_kernel(const float *__restrict__ a, const float *__restrict__ b, int64_t n,
                           float *__restrict__ grad, double *__restrict__ part)
{
    __shared__ double sh[256];
    double acc = 0.0;
    const float sc = 2.0f / (float)n;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float dlt = a[i] - b[i];
        grad[i] = sc * dlt;
        acc += (double)dlt * dlt;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int t = 0; t < (int)blockDim.x; ++t) s += sh[t];
        part[blockIdx.x] = s;
    }
}

__global__ void sum_partials_f64(const double *__restrict__ part, int n, double scale, double *__restrict__ out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += part[i];
        *out = s * scale;
    }
}

// Adam on FP32 master weights, with a BF16 copy for the kernels (optional)
__global__ void adam_kernel(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                            float *__restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                            float c1, float c2, __bf16 *__restrict__ pb)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float upd = lr * (mi * c1) / (sqrtf(vi * c2) + eps);
        const float np = p[i] - upd;
        p[i] = np;
        if (pb) pb[i] = (__bf16)np;
    }
}

}  // namespace cvpnn

// ------------------------------------------------------------------ C ABI
#include "cvp.h"

namespace {

cvpnn::Act act(const cvp_nn_tensor *t)
{
    cvpnn::Act a;
    a.p = reinterpret_cast<__bf16 *>(t->data);
    a.D = t->d; a.H = t->h; a.W = t->w; a.C = t->channels; a.stride = t->stride;
    return a;
}

bool valid(const cvp_nn_tensor *t)
{
    return t && t->data && t->d > 0 && t->h > 0 && t->w > 0 && t->channels > 0 &&
           t->stride >= t->channels && (t->channels % 8) == 0 && (t->stride % 8) == 0 &&
           (reinterpret_cast<uintptr_t>(t->data) & 15) == 0;
}

cvp_status st(hipError_t e) { return e == hipSuccess ? CVP_OK : CVP_E_DEVICE; }

int grid_for(int64_t n) { return (int)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096); }

// The LDS-tiled convolutions take more than the default 64 KB of dynamic LDS
// (32 or 64 input channels: 76 or 78 KB); allowed once per process.
hipError_t conv_lds_setup()
{
    static hipError_t done = [] {
        hipError_t e = hipSuccess;
#define ALLOW(CO_, CI_, RX_)                                                                                 \
        if (e == hipSuccess)                                                                                 \
            e = hipFuncSetAttribute(reinterpret_cast<const void *>(cvpnn::conv3d_lds_kernel<CO_, CI_, RX_>), \
                                    hipFuncAttributeMaxDynamicSharedMemorySize,                              \
                                    cvpnn::conv_tile_bytes<CI_, RX_>());
        ALLOW(16, 16, 4) ALLOW(16, 32, 4) ALLOW(32, 16, 4) ALLOW(32, 32, 4) ALLOW(64, 32, 4)
        ALLOW(16, 16, 2) ALLOW(16, 32, 2) ALLOW(16, 64, 2) ALLOW(32, 16, 2) ALLOW(32, 32, 2) ALLOW(32, 64, 2)
        ALLOW(64, 32, 2) ALLOW(64, 64, 2)
#undef ALLOW
        return e;
    }();
    return done;
}

}  // namespace

extern "C" {

cvp_status cvp_nn_conv3d(const cvp_nn_tensor *in, const void *weight, const float *bias,
                         const cvp_nn_tensor *out, int32_t relu, int32_t flip, void *stream)
{
    if (!valid(in) || !valid(out) || !weight) return CVP_E_INVALID;
    if (in->d != out->d || in->h != out->h || in->w != out->w) return CVP_E_INVALID;
    const cvpnn::Act a = act(in), o = act(out);
    const int rows = in->d * in->h * ((in->w + 63) / 64);
    const dim3 grid((rows + 3) / 4), block(256);
    hipStream_t s = (hipStream_t)stream;
    const __bf16 *w = reinterpret_cast<const __bf16 *>(weight);
    // channel counts 16, 32, 64 and 32-bit element offsets: the specialised kernel
    const int64_t elems = (int64_t)in->d * in->h * in->w * std::max(in->stride, out->stride);
    const int ci = in->channels, co = out->channels;
    const bool spec = elems < (int64_t(1) << 31) && (ci == 16 || ci == 32 || ci == 64);
#define CONVC(CO_, CI_) hipLaunchKernelGGL((cvpnn::conv3d_kernel_c<CO_, CI_>), grid, block, 0, s, a, w, bias, o, relu, flip)
    // the LDS-tiled kernel (4 rows of a slice per workgroup): 64-voxel rows
    // with 16 or 32 input channels, 32-voxel rows with 64 (a 78 KB tile; at
    // 32^3 with 32 channels the 64-voxel rows were faster, 35 against 49 us)
    const int rx = ci == 64 ? 2 : 4;
    const dim3 lgrid(in->d * ((in->h + 3) / 4) * ((in->w + rx * 16 - 1) / (rx * 16)));
#define CONVL(CO_, CI_, RX_) hipLaunchKernelGGL((cvpnn::conv3d_lds_kernel<CO_, CI_, RX_>), lgrid, block, \
                                                (cvpnn::conv_tile_bytes<CI_, RX_>()), s, a, w, bias, o, relu, flip)
    if (spec) {
        const hipError_t e = conv_lds_setup();
        if (e != hipSuccess) return st(e);
    }
    if (spec && co == 64 && ci == 16) CONVC(64, 16);   // the LDS kernel's registers would spill
    else if (spec && rx == 4 && co == 16 && ci == 16) CONVL(16, 16, 4);
    else if (spec && rx == 4 && co == 16 && ci == 32) CONVL(16, 32, 4);
    else if (spec && rx == 4 && co == 32 && ci == 16) CONVL(32, 16, 4);
    else if (spec && rx == 4 && co == 32 && ci == 32) CONVL(32, 32, 4);
    else if (spec && rx == 4 && co == 64 && ci == 32) CONVL(64, 32, 4);
    else if (spec && co == 16 && ci == 16) CONVL(16, 16, 2);
    else if (spec && co == 16 && ci == 32) CONVL(16, 32, 2);
    else if (spec && co == 16 && ci == 64) CONVL(16, 64, 2);
    else if (spec && co == 32 && ci == 16) CONVL(32, 16, 2);
    else if (spec && co == 32 && ci == 32) CONVL(32, 32, 2);
    else if (spec && co == 32 && ci == 64) CONVL(32, 64, 2);
    else if (spec && co == 64 && ci == 32) CONVL(64, 32, 2);
    else if (spec && co == 64 && ci == 64) CONVL(64, 64, 2);
    else {
        switch (co) {
        case 16: hipLaunchKernelGGL(cvpnn::conv3d_kernel<16>, grid, block, 0, s, a, w, bias, o, relu, flip); break;
        case 32: hipLaunchKernelGGL(cvpnn::conv3d_kernel<32>, grid, block, 0, s, a, w, bias, o, relu, flip); break;
        case 64: hipLaunchKernelGGL(cvpnn::conv3d_kernel<64>, grid, block, 0, s, a, w, bias, o, relu, flip); break;
        default: return CVP_E_UNSUPPORTED;
        }
    }
#undef CONVC
#undef CONVL
    return st(hipGetLastError());
}

cvp_status cvp_nn_wgrad_workspace(const cvp_nn_tensor *x, const cvp_nn_tensor *dy, int64_t *floats)
{
    if (!x || !dy || !floats) return CVP_E_INVALID;
    const int rows = x->d * x->h;
    const int chunks = (rows + 63) / 64;
    *floats = (int64_t)chunks * 27 * dy->channels * x->channels;
    return CVP_OK;
}

cvp_status cvp_nn_conv3d_wgrad(const cvp_nn_tensor *x, const cvp_nn_tensor *dy, float *dw, float *work,
                               int64_t work_floats, void *stream)
{
    if (!valid(x) || !valid(dy) || !dw || !work) return CVP_E_INVALID;
    int64_t need = 0;
    cvp_nn_wgrad_workspace(x, dy, &need);
    if (work_floats < need) return CVP_E_INVALID;
    const cvpnn::Act a = act(x), g = act(dy);
    const int rows = x->d * x->h, rpc = 64, chunks = (rows + rpc - 1) / rpc;
    const dim3 grid(chunks, 9), block(256);
    hipStream_t s = (hipStream_t)stream;
    const int co = dy->channels, ci = x->channels;
#define WG(CO_, CI_) hipLaunchKernelGGL((cvpnn::conv3d_wgrad_kernel<CO_, CI_>), grid, block, 0, s, a, g, rpc, work)
    if (co == 16 && ci == 16) WG(16, 16);
    else if (co == 16 && ci == 32) WG(16, 32);
    else if (co == 32 && ci == 16) WG(32, 16);
    else if (co == 32 && ci == 32) WG(32, 32);
    else if (co == 32 && ci == 64) WG(32, 64);
    else if (co == 64 && ci == 32) WG(64, 32);
    else if (co == 64 && ci == 64) WG(64, 64);
    else if (co == 16 && ci == 64) WG(16, 64);
    else return CVP_E_UNSUPPORTED;
#undef WG
    const int64_t n = (int64_t)27 * co * ci;
    hipLaunchKernelGGL(cvpnn::reduce_chunks, dim3(grid_for(4 * n)), dim3(256), 0, s, work, chunks, n, dw);
    return st(hipGetLastError());
}

cvp_status cvp_nn_channel_sum(const cvp_nn_tensor *a, float *out, float *work, int64_t work_floats,
                              void *stream)
{
    if (!valid(a) || !out || !work) return CVP_E_INVALID;
    if (a->channels > 2048) return CVP_E_UNSUPPORTED;
    const int rows = a->d * a->h, rpc = 16, chunks = (rows + rpc - 1) / rpc;
    if (work_floats < (int64_t)chunks * a->channels) return CVP_E_INVALID;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(cvpnn::channel_sum_partials, dim3(chunks), dim3(256), 0, s, act(a), rpc, work);
    hipLaunchKernelGGL(cvpnn::reduce_chunks, dim3(1), dim3(256), 0, s, work, chunks, (int64_t)a->channels, out);
    return st(hipGetLastError());
}

cvp_status cvp_nn_relu_mask(const cvp_nn_tensor *dy, const cvp_nn_tensor *y, void *stream)
{
    if (!valid(dy) || !valid(y)) return CVP_E_INVALID;
    const int64_t n = (int64_t)dy->d * dy->h * dy->w * dy->channels / 8;
    if (n < (int64_t(1) << 31))
        hipLaunchKernelGGL(cvpnn::relu_mask<int>, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, act(dy), act(y));
    else
        hipLaunchKernelGGL(cvpnn::relu_mask<int64_t>, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, act(dy),
                           act(y));
    return st(hipGetLastError());
}

static cvp_status resample(int kind, const cvp_nn_tensor *a, const cvp_nn_tensor *b, void *stream)
{
    if (!valid(a) || !valid(b) || a->channels != b->channels) return CVP_E_INVALID;
    hipStream_t s = (hipStream_t)stream;
    const cvp_nn_tensor *big = (kind == 0 || kind == 3) ? a : b;    // fine-resolution operand
    const cvp_nn_tensor *small = big == a ? b : a;
    if (big->d != 2 * small->d || big->h != 2 * small->h || big->w != 2 * small->w) return CVP_E_INVALID;
    // 8-channel chunks of the fine and the coarse operand
    const int64_t nb = (int64_t)big->d * big->h * big->w * big->channels / 8;
    const int64_t ns = nb / 8;
    const bool i32 = nb < (int64_t(1) << 31);
#define RS(K, N)                                                                                      \
    do {                                                                                              \
        if (i32) hipLaunchKernelGGL(cvpnn::K<int>, dim3(grid_for(N)), dim3(256), 0, s, act(a), act(b)); \
        else hipLaunchKernelGGL(cvpnn::K<int64_t>, dim3(grid_for(N)), dim3(256), 0, s, act(a), act(b)); \
    } while (0)
    switch (kind) {
    case 0: RS(avgpool2, ns); break;
    case 1: RS(avgpool2_bwd, nb); break;
    case 2: RS(upsample2, nb); break;
    default: RS(upsample2_bwd, ns); break;
    }
#undef RS
    return st(hipGetLastError());
}

cvp_status cvp_nn_avgpool2(const cvp_nn_tensor *in, const cvp_nn_tensor *out, void *stream) { return resample(0, in, out, stream); }
cvp_status cvp_nn_avgpool2_bwd(const cvp_nn_tensor *dout, const cvp_nn_tensor *din, void *stream) { return resample(1, dout, din, stream); }
cvp_status cvp_nn_upsample2(const cvp_nn_tensor *in, const cvp_nn_tensor *out, void *stream) { return resample(2, in, out, stream); }
cvp_status cvp_nn_upsample2_bwd(const cvp_nn_tensor *dout, const cvp_nn_tensor *din, void *stream) { return resample(3, dout, din, stream); }

cvp_status cvp_nn_add(const cvp_nn_tensor *a, const cvp_nn_tensor *b, const cvp_nn_tensor *out, void *stream)
{
    if (!valid(a) || !valid(b) || !valid(out) || a->channels != out->channels || b->channels != out->channels ||
        a->d != out->d || a->h != out->h || a->w != out->w || b->d != out->d || b->h != out->h || b->w != out->w)
        return CVP_E_INVALID;
    const int64_t n = (int64_t)out->d * out->h * out->w * out->channels / 8;
    if (n < (int64_t(1) << 31))
        hipLaunchKernelGGL(cvpnn::add_kernel<int>, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, act(a), act(b),
                           act(out));
    else
        hipLaunchKernelGGL(cvpnn::add_kernel<int64_t>, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, act(a),
                           act(b), act(out));
    return st(hipGetLastError());
}

cvp_status cvp_nn_transpose_weights(const void *w, void *wt, int32_t co, int32_t ci, void *stream)
{
    if (!w || !wt || co <= 0 || ci <= 0) return CVP_E_INVALID;
    const int64_t n = (int64_t)27 * co * ci;
    hipLaunchKernelGGL(cvpnn::transpose_weights, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream,
                       reinterpret_cast<const __bf16 *>(w), reinterpret_cast<__bf16 *>(wt), co, ci);
    return st(hipGetLastError());
}

cvp_status cvp_nn_pack_input(const float *x1, const float *x2, float scale, const cvp_nn_tensor *out, void *stream)
{
    if (!x1 || !x2 || !valid(out) || out->channels != 16) return CVP_E_INVALID;
    const int64_t n = (int64_t)out->d * out->h * out->w;
    hipLaunchKernelGGL(cvpnn::pack_input, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, x1, x2, n, scale, act(out));
    return st(hipGetLastError());
}

cvp_status cvp_nn_head(const cvp_nn_tensor *h, const float *w, const float *b, const float *x2, float scale,
                       float *x0, void *stream)
{
    if (!valid(h) || h->channels > 16 || !w || !b || !x2 || !x0 || !(scale > 0)) return CVP_E_INVALID;
    const int64_t n = (int64_t)h->d * h->h * h->w;
    hipLaunchKernelGGL(cvpnn::head_fwd, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, act(h), w, b, x2,
                       1.0f / scale, x0);
    return st(hipGetLastError());
}

cvp_status cvp_nn_head_bwd(const cvp_nn_tensor *h, const float *w, const float *g, float scale,
                           const cvp_nn_tensor *dh, float *dwb /*17*/, float *work, int64_t work_floats,
                           void *stream)
{
    if (!valid(h) || !valid(dh) || h->channels > 16 || !w || !g || !dwb || !work || !(scale > 0)) return CVP_E_INVALID;
    const int64_t n = (int64_t)h->d * h->h * h->w;
    const int64_t per = 4096;
    const int blocks = (int)((n + per - 1) / per);
    if (work_floats < (int64_t)blocks * 17) return CVP_E_INVALID;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(cvpnn::head_bwd, dim3(blocks), dim3(256), 0, s, act(h), w, g, 1.0f / scale, act(dh), per, work);
    hipLaunchKernelGGL(cvpnn::reduce_chunks, dim3(1), dim3(256), 0, s, work, blocks, (int64_t)17, dwb);
    return st(hipGetLastError());
}

cvp_status cvp_nn_mse(const float *a, const float *b, int64_t n, float *grad, double *loss, double *work,
                      int64_t work_doubles, void *stream)
{
    if (!a || !b || !grad || !loss || !work || n <= 0 || work_doubles < 1024) return CVP_E_INVALID;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(cvpnn::mse_kernel, dim3(1024), dim3(256), 0, s, a, b, n, grad, work);
    hipLaunchKernelGGL(cvpnn::sum_partials_f64, dim3(1), dim3(64), 0, s, work, 1024, 1.0 / (double)n, loss);
    return st(hipGetLastError());
}

cvp_status cvp_nn_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr, float beta1,
                       float beta2, float eps, int32_t step, void *p_bf16, void *stream)
{
    if (!p || !g || !m || !v || n <= 0 || step < 1) return CVP_E_INVALID;
    const float c1 = 1.0f / (1.0f - powf(beta1, (float)step));
    const float c2 = 1.0f / (1.0f - powf(beta2, (float)step));
    hipLaunchKernelGGL(cvpnn::adam_kernel, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, p, g, m, v, n, lr,
                       beta1, beta2, eps, c1, c2, reinterpret_cast<__bf16 *>(p_bf16));
    return st(hipGetLastError());
}

}  // extern "C"
