// Cutting voxel projector kernels for gfx950 (MI355X).
//
// Kulvait & Rose, "Cutting Voxel Projector a New Approach to Construct 3D Cone
// Beam CT Operator" (2021).  Both directions apply the same weights
//   w = mu * |V^(ijk)_(uv)| / r^2            (Sec. II-F, eq. vox)
// with the cut volume estimated as A_u * d_uv (Sec. III-A, eq. cutvolume) and
// the per-pixel factor sigma_uv applied to the unscaled sums (eq. cvpsu).
//
// Work split (one launch per direction, no global atomics):
//  * projection: a workgroup owns one view and a band of U detector columns.
//    It walks every voxel column whose base meets the band's wedge (by the
//    column identity of Sec. III-A the wedge is the same for all k), computes
//    the column cut pieces once per column in FP64, and then, with lanes over
//    k, scatters each voxel's row pieces, rounded to integers, into a 64-bit
//    fixed-point band image in LDS with integer atomics (scale chosen per
//    work item from the largest |mu| in its wedge, read from per-group maxima
//    when the caller gives scratch).  The band is written once at the end,
//    scaled by sigma.  Integer sums make the result independent of the order
//    of the additions (scheduling, the wave split, batching).
//  * backprojection: a workgroup owns a stack of GW columns x 64 kp voxels;
//    each wave takes every 4th view, builds the stack's piece records (for
//    several views per pass when the stack is narrow), stages the
//    pre-scaled detector window in LDS and gathers into registers.  Each
//    voxel is written once, and its sum does not depend on the plan.
//
// Numerics: the column stage (polygon moments, centroid depth) runs in FP64
// (the rate of unpacked FP32 on CDNA4); the per-voxel stage runs in FP32 on quantities
// that are small by construction: detector row positions are split into a
// 2^-10-quantised high part, whose differences with half-integer row
// boundaries are exact, plus a small low part.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>
#include <type_traits>

#include "cvp_internal.h"

namespace cvp {
namespace {

// No implicit FP contraction anywhere in this file: a multiply-add is fused
// only where the source says fmaf/fma.  Otherwise the compiler may fuse
// differently in each kernel a device function is inlined into, and the
// single-problem and batched launches would not give the same bits.
#pragma clang fp contract(off)

// ------------------------------------------------------------ FP64 column stage
// FP contraction is off in this stage, so the records do not depend on the
// kernel the stage is inlined into (single-problem and batched launches give
// the same bits).

// Shoelace sums of a polygon: a2 = 2A, sx = 6A cx, sy = 6A cy,
// sxx = 12 int x^2, syy = 12 int y^2, sxy = 24 int xy.
struct Mom {
    double a2, sx, sy, sxx, sxy, syy;
};

__device__ __forceinline__ void mom_edge(Mom &m, double x0, double y0, double x1, double y1)
{
#pragma clang fp contract(off)
    const double cr = x0 * y1 - x1 * y0;
    m.a2 += cr;
    m.sx += (x0 + x1) * cr;
    m.sy += (y0 + y1) * cr;
    m.sxx += (x0 * x0 + x0 * x1 + x1 * x1) * cr;
    m.syy += (y0 * y0 + y0 * y1 + y1 * y1) * cr;
    m.sxy += (x0 * y1 + 2.0 * x0 * y0 + 2.0 * x1 * y1 + x1 * y0) * cr;
}

// Moments of the square [-h1,h1] x [-h2,h2] cut to {q : gx qx + gy qy + c <= 0}
// by Green's theorem: the inside parts of the square's edges (counter-
// clockwise) plus the chord along the cutting line from exit to entry.
__device__ __forceinline__ Mom halfplane_moments(double h1, double h2, double gx, double gy,
                                                 double c)
{
#pragma clang fp contract(off)
    const double px[4] = {-h1, h1, h1, -h1};
    const double py[4] = {-h2, -h2, h2, h2};
    double val[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) val[k] = gx * px[k] + gy * py[k] + c;
    Mom m = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    double ex = 0.0, ey = 0.0, nx = 0.0, ny = 0.0;
    bool has_exit = false, has_entry = false;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int b = (k + 1) & 3;
        const double va = val[k], vb = val[b];
        if (va <= 0.0 && vb <= 0.0) {
            mom_edge(m, px[k], py[k], px[b], py[b]);
        } else if (va <= 0.0) {
            const double t = va / (va - vb);
            const double xx = px[k] + t * (px[b] - px[k]), yy = py[k] + t * (py[b] - py[k]);
            mom_edge(m, px[k], py[k], xx, yy);
            ex = xx; ey = yy; has_exit = true;
        } else if (vb <= 0.0) {
            const double t = va / (va - vb);
            const double xx = px[k] + t * (px[b] - px[k]), yy = py[k] + t * (py[b] - py[k]);
            mom_edge(m, xx, yy, px[b], py[b]);
            nx = xx; ny = yy; has_entry = true;
        }
    }
    if (has_exit && has_entry) mom_edge(m, ex, ey, nx, ny);
    return m;
}

// One voxel column (i, j) seen from one view.  Local coordinates q are
// relative to the column centre.  chi1(x) <= t  <=>  G(t).q + chi1c - t <= 0
// with G(t) = ((f/b1) e1 - (t - c1) d) / Dc: the half-plane of the paper's
// polygons H- / H+ (Sec. III-A), normalised by the centre depth Dc > 0.
struct Column {
    double xc1, xc2;   // centre
    double Dc;         // depth of the centre, d.(xc - s)
    double iDc;        // 1 / Dc
    double chic;       // chi1 of the centre
    double chimin, chimax;
};

__device__ __forceinline__ Column make_column(const DevGeom &G, const ViewGeom &V, int i, int j)
{
#pragma clang fp contract(off)
    Column C;
    C.xc1 = G.x1lo + (i + 0.5) * G.a1;
    C.xc2 = G.x2lo + (j + 0.5) * G.a2;
    const double r1 = C.xc1 - V.s1, r2 = C.xc2 - V.s2;
    const double P1 = V.e1x * r1 + V.e1y * r2;
    C.Dc = V.dx * r1 + V.dy * r2;
    C.iDc = 1.0 / C.Dc;
    const double fb = V.fb1;
    C.chic = V.c1 + fb * P1 * C.iDc;
    double mn = 1e300, mx = -1e300;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double q1 = (k & 1) ? 0.5 * G.a1 : -0.5 * G.a1;
        const double q2 = (k & 2) ? 0.5 * G.a2 : -0.5 * G.a2;
        const double ch = V.c1 + fb * (P1 + V.e1x * q1 + V.e1y * q2) / (C.Dc + V.dx * q1 + V.dy * q2);
        mn = fmin(mn, ch);
        mx = fmax(mx, ch);
    }
    C.chimin = mn;
    C.chimax = mx;
    return C;
}

__device__ __forceinline__ Mom column_prefix(const DevGeom &G, const ViewGeom &V, const Column &C,
                                             double t)
{
#pragma clang fp contract(off)
    const double fb = V.fb1;
    const double inv = C.iDc;
    const double gx = (fb * V.e1x - (t - V.c1) * V.dx) * inv;
    const double gy = (fb * V.e1y - (t - V.c1) * V.dy) * inv;
    return halfplane_moments(0.5 * G.a1, 0.5 * G.a2, gx, gy, C.chic - t);
}

// Record of one cut piece H_u for the FP32 voxel stage (12 floats):
//  [0] u (int bits)  [1] W = A_u * b2 D_u / f       [2] Y0 hi   [3] Y0 lo
//  [4] beta hi       [5] beta lo   [6] beta          [7] rho = h/D (EC)
//  [8] R^2 of the column centre (x1x2 part of r^2, relaxed form)
//  [9] b2 D_u / f (mm of x3 per row)  [10] EC row margin factor
//  [11] R^2 of the cut centroid (exact form)
// Y(k) = Y0 - k beta is chi2 of the top face of voxel k at the centroid depth.
// lo / hi: column_prefix at u - 1/2 and u + 1/2.  The record is the same for
// every option (the kernels read the slots their form needs), so a geometry's
// table of records serves them all.
template <bool EXACT, bool EC>
__device__ __forceinline__ void piece_record(const DevGeom &G, const ViewGeom &V, const Column &C,
                                             int u, const Mom &lo, const Mom &hi, float *rec)
{
#pragma clang fp contract(off)
    const double a2 = hi.a2 - lo.a2;
    const double A = 0.5 * a2;
    double cx = 0.0, cy = 0.0, var = 0.0;
    if (A > 1e-12 * G.a1 * G.a2) {
        // one division: 1/(3 a2), 1/(12 A) = 2/(3 a2), 1/(24 A) = 1/(3 a2)
        const double i3 = 1.0 / (3.0 * a2);
        cx = (hi.sx - lo.sx) * i3;
        cy = (hi.sy - lo.sy) * i3;
        const double cxx = (hi.sxx - lo.sxx) * (0.5 * i3) - cx * cx;
        const double cyy = (hi.syy - lo.syy) * (0.5 * i3) - cy * cy;
        const double cxy = (hi.sxy - lo.sxy) * (0.25 * i3) - cx * cy;
        var = V.dx * V.dx * cxx + 2.0 * V.dx * V.dy * cxy + V.dy * V.dy * cyy;
        if (!(var > 0.0)) var = 0.0;
    }
    const double Du = C.Dc + V.dx * cx + V.dy * cy;
    const double iDu = 1.0 / Du;
    const double gmm = V.ifb2 * Du;              // x3 mm per detector row at depth Du
    const double ig = V.fb2 * iDu;
    const double Y0 = V.c2 - (G.x3lo + G.a3 - V.s3) * ig;
    const double beta = G.a3 * ig;
    const double Y0h = rint(Y0 * 1024.0) * (1.0 / 1024.0);
    const double bh = rint(beta * 1024.0) * (1.0 / 1024.0);
    const double p1 = C.xc1 + cx - V.s1, p2 = C.xc2 + cy - V.s2;   // cut centroid
    const double q1 = C.xc1 - V.s1, q2 = C.xc2 - V.s2;             // column centre
    rec[0] = __int_as_float(u);
    rec[1] = (A > 1e-12 * G.a1 * G.a2) ? (float)(A * gmm) : 0.0f;
    rec[2] = (float)Y0h;
    rec[3] = (float)(Y0 - Y0h);
    rec[4] = (float)bh;
    rec[5] = (float)(beta - bh);
    rec[6] = (float)beta;
    rec[7] = (float)(sqrt(3.0 * var) * iDu);
    rec[8] = (float)(q1 * q1 + q2 * q2);
    rec[9] = (float)gmm;
    // EC row margin factor 1.01 rho / (1 - rho) from the FP32 rho the voxel
    // stage uses (see row_range_unclipped)
    const double rho32 = (double)rec[7];
    rec[10] = (float)(1.01 * rho32 / fmax(1.0 - rho32, 0.05));
    rec[11] = (float)(p1 * p1 + p2 * p2);
}

// Record of the TT separable footprint (the footprint projector the paper
// compares with, Sec. I and IV: Long, Fessler & Balter 2010) of column C at
// detector column u, in the slots of piece_record:
//  [0] u (int bits)  [1] F1(u) min(a1/|r1|, a2/|r2|)  [2] Y0 hi  [3] Y0 lo
//  [4] beta hi  [5] beta lo  [6] beta  [7] rho = (Df - Dn) / (Df + Dn)
//  [8] R^2 = |r_xy|^2 of the column centre  [9] 0  [10] row margin 1.01 rho
// F1(u) integrates over [u - 1/2, u + 1/2] the height-1 trapezoid whose
// vertices are the sorted chi1 of the four base corners (the transaxial
// footprint).  The axial footprint of voxel k is the trapezoid between the
// chi2 of its top and bottom faces at the nearest (Dn) and farthest (Df)
// depth of the base: Y(k) = Y0 - k beta is the middle of the top face's
// ramp, Y(k) + beta that of the bottom face, and a face at Y has the ramp
// half-width |Y - c2| rho.  The amplitude is the central ray's chord,
// min(a1/|r1|, a2/|r2|) |r| with r = centre - s; its |r| is applied per
// voxel.  FP64 like the rest of the column stage.
__device__ __forceinline__ void tt_record(const DevGeom &G, const ViewGeom &V, const Column &C, int u, float *rec)
{
#pragma clang fp contract(off)
    const double r1 = C.xc1 - V.s1, r2 = C.xc2 - V.s2;
    const double P1 = V.e1x * r1 + V.e1y * r2;
    double t[4], Dn = 1e300, Df = -1e300;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double q1 = (k & 1) ? 0.5 * G.a1 : -0.5 * G.a1;
        const double q2 = (k & 2) ? 0.5 * G.a2 : -0.5 * G.a2;
        const double D = C.Dc + V.dx * q1 + V.dy * q2;
        t[k] = V.c1 + V.fb1 * (P1 + V.e1x * q1 + V.e1y * q2) / D;
        Dn = fmin(Dn, D);
        Df = fmax(Df, D);
    }
    // sort the four vertices (a five-exchange network)
    auto cx = [&](int a, int b) {
        const double lo = fmin(t[a], t[b]), hi = fmax(t[a], t[b]);
        t[a] = lo;
        t[b] = hi;
    };
    cx(0, 1); cx(2, 3); cx(0, 2); cx(1, 3); cx(1, 2);
    // the trapezoid's integral up to x: rise minus fall, each a hinge
    // smoothed over its ramp (middle m, half-width e)
    auto hinge = [](double x, double m, double e) {
        const double p = fmax(e - fabs(x - m), 0.0);
        return fmax(x - m, 0.0) + (e > 0.0 ? p * p / (4.0 * e) : 0.0);
    };
    const double mu = 0.5 * (t[0] + t[1]), eu = 0.5 * (t[1] - t[0]);
    const double md = 0.5 * (t[2] + t[3]), ed = 0.5 * (t[3] - t[2]);
    const double F1 = (hinge(u + 0.5, mu, eu) - hinge(u + 0.5, md, ed)) - (hinge(u - 0.5, mu, eu) - hinge(u - 0.5, md, ed));
    const double lphi = fmin(G.a1 / fabs(r1), G.a2 / fabs(r2));
    const double in = 1.0 / Dn, ifar = 1.0 / Df;
    const double ig = 0.5 * V.fb2 * (in + ifar);
    const double Y0 = V.c2 - (G.x3lo + G.a3 - V.s3) * ig;
    const double beta = G.a3 * ig;
    const double Y0h = rint(Y0 * 1024.0) * (1.0 / 1024.0);
    const double bh = rint(beta * 1024.0) * (1.0 / 1024.0);
    const double rho = (in - ifar) / (in + ifar);
    rec[0] = __int_as_float(u);
    rec[1] = (float)(F1 * lphi);
    rec[2] = (float)Y0h;
    rec[3] = (float)(Y0 - Y0h);
    rec[4] = (float)bh;
    rec[5] = (float)(beta - bh);
    rec[6] = (float)beta;
    rec[7] = (float)rho;
    rec[8] = (float)(r1 * r1 + r2 * r2);
    rec[9] = 0.0f;
    rec[10] = (float)(1.01 * rho);
    rec[11] = 0.0f;
}

// ------------------------------------------------------------ FP32 voxel stage

// Row weights.  The voxel's chi2 extent is [Ytop, Ybot] (Ybot = Ytop + beta)
// and row v covers [t, t + 1], t = v - 1/2.  With s1 = Ytop - t and
// s0 = Ybot - t the plain x3 share of the row is the overlap
//   m(t) = med3(s0, 0, 1) - med3(s1, 0, 1)
// (Sec. III-A).  With the elevation correction each row boundary moves
// uniformly over [t - e, t + e], e = |t - c2| h / D (Sec. III-B reading); the
// box average of max(s, 0) is max(s, 0) + max(e - |s|, 0)^2 / (4e), so the
// row gets m(t) + Phi(t) - Phi(t + 1) with
//   Phi(t) = (p0^2 - p1^2) / (4e),  p = max(e - |s|, 0)
// at each boundary.  Every term is a small number computed from the face
// offsets near that face: s1 = d + Yl and s0 = d0 + Ybl with d = Ytop_hi - t
// and d0 = Ybot_hi - t exact (high parts on a 2^-10 grid) and Yl, Ybl the low
// parts, so a thin sliver at either face keeps its relative precision however
// many rows tall the voxel is, and a row the box average does not reach gets
// exactly 0 (m = 0 and Phi = 0 at both its boundaries).
// rho4 = 4 rho; 1/(4e) is taken of 4e + 1e-30, which only differs from 4e
// where e = 0, and there p0 = p1 = 0.
template <bool EC>
__device__ __forceinline__ void boundary(float d, float Yl, float d0, float Ybl, float tc, float rho, float rho4,
                                         float &s1, float &m, float &phi)
{
    s1 = d + Yl;
    const float s0 = d0 + Ybl;
    m = __builtin_amdgcn_fmed3f(s0, 0.0f, 1.0f) - __builtin_amdgcn_fmed3f(s1, 0.0f, 1.0f);
    phi = 0.0f;
    if (EC) {
        const float p0 = fmaxf(fmaf(fabsf(tc), rho, -fabsf(s0)), 0.0f);
        const float p1 = fmaxf(fmaf(fabsf(tc), rho, -fabsf(s1)), 0.0f);
        const float inv4e = __builtin_amdgcn_rcpf(fmaf(fabsf(tc), rho4, 1e-30f));
        phi = fmaf(p0, p0, -(p1 * p1)) * inv4e;
    }
}

// Row weights of the TT axial footprint: the trapezoid that rises over the
// top face's ramp (middle Ytop, half-width eu) and falls over the bottom
// face's (middle Ybot, half-width ed).  Its integral over row [t, t + 1] is
// m(t) + Phi(t) - Phi(t + 1): m the overlap of [Ytop, Ybot] with the row as
// in boundary, and Phi(t) = p0^2 / (4 ed) - p1^2 / (4 eu), p = max(e - |s|,
// 0), each ramp a hinge smoothed over its width.  iu = 1 / (4 eu), id =
// 1 / (4 ed); FULL = false gives m alone (Phi = 0 where no ramp reaches t).
template <bool FULL>
__device__ __forceinline__ void boundary_tt(float d, float Yl, float d0, float Ybl, float eu, float ed, float iu,
                                            float id, float &s1, float &m, float &phi)
{
    s1 = d + Yl;
    const float s0 = d0 + Ybl;
    m = __builtin_amdgcn_fmed3f(s0, 0.0f, 1.0f) - __builtin_amdgcn_fmed3f(s1, 0.0f, 1.0f);
    phi = 0.0f;
    if (FULL) {
        const float p0 = fmaxf(ed - fabsf(s0), 0.0f);
        const float p1 = fmaxf(eu - fabsf(s1), 0.0f);
        phi = fmaf(p0 * p0, id, -((p1 * p1) * iu));
    }
}

// Fixed-point accumulation of the projection.  A contribution w, already
// scaled by the work item's 2^s so that |w| < 2^51, becomes a 64-bit integer
// by one FP64 addition: w + 1.5 * 2^52 lies in [2^52, 2^53), where the FP64
// spacing is 1, so the addition rounds w to the nearest integer (ties to
// even) and the low 52 bits of the result hold that integer plus 2^51; the
// bit pattern minus that of 1.5 * 2^52 (whose low word is zero, so only the
// high word changes) is the integer in two's complement.  It is added with
// an integer LDS atomic; the 64-bit sums hold a pixel's total.  On gfx950
// the integer atomic is about thirty times cheaper than ds_add_f32, and
// integer sums do not depend on the order of the additions.
__device__ __forceinline__ void lds_add_fixed(unsigned long long *p, float w)
{
    const double d = (double)w + 0x1.8p52;
    const unsigned hi = (unsigned)__double2hiint(d) - 0x43380000u;
    const unsigned lo = (unsigned)__double2loint(d);
    const unsigned long long q = ((unsigned long long)hi << 32) | lo;
    __hip_atomic_fetch_add(p, q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ double fixed_to_double(unsigned long long q)
{
    return (double)(int)(unsigned)(q >> 32) * 0x1p32 + (double)(unsigned)q;
}

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Row range of a piece, before clipping to the detector: the rows its chi2
// extent [Ytop, Ytop + beta] touches, widened by 1e-3 for FP32 rounding and,
// with EC, by a margin E at least the box half-width e(t) = |t - c2| rho at
// every boundary t within a row of the extent, i.e. E (1 - rho) >= rho
// (max |Y - c2| + 1.001).  Then the range covers every row the box average
// reaches, and C is exactly beta / 0 at its first / last boundary.  Valid
// for rho < 0.9 (a box narrower than the source distance).  mfac = 1.01 rho
// / max(1 - rho, 0.05) comes with the piece record; E = mfac (M + 1.01) with
// M = max(|Ytop - c2|, |Ytop + beta - c2|) = max(Ytop + beta - c2, c2 - Ytop).
__device__ __forceinline__ int floor_to_int(float x)
{
    int r;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

template <bool EC>
__device__ __forceinline__ void row_range_unclipped(float Ytop, float beta, float mfac, float c2f, int &vlo0,
                                                    int &vhi0)
{
    const float yb = Ytop + beta;
    float lo = Ytop + 0.499f, hi = yb + 0.501f;
    if (EC) {
        const float M1 = fmaxf(yb - c2f, c2f - Ytop) + 1.01f;
        lo = fmaf(-mfac, M1, lo);
        hi = fmaf(mfac, M1, hi);
    }
    vlo0 = floor_to_int(lo);
    vhi0 = floor_to_int(hi);
}

// The same range clipped to the detector rows [0, N - 1].
template <bool EC>
__device__ __forceinline__ void row_range(float Ytop, float beta, float mfac, float c2f, int N, int &vlo,
                                          int &vhi)
{
    row_range_unclipped<EC>(Ytop, beta, mfac, c2f, vlo, vhi);
    vlo = max(vlo, 0);
    vhi = min(vhi, N - 1);
}

// Row weights of one voxel piece: rows [vlo, vhi] (already clipped) of the
// unclipped range [vlo0, vhi0], added to the band column bcol.  The unclipped
// range includes the EC margin, so Phi is exactly 0 at its first and last
// boundaries; those two box averages are skipped unless clipping moved the
// boundary.  Boundaries t = vlo - 1/2, vlo + 1/2, ...: d, d0 step by exactly
// 1; tc = t - c2 feeds only the box width.  Weight of row [t, t + 1]:
// coef (m(t) + Phi(t) - Phi(t + 1)).  The bottom face's high part is Yh + bh
// (bh the high part of one slice's step).
template <bool EC, bool EXACT>
__device__ __forceinline__ void sweep_rows(int vlo0, int vhi0, int vlo, int vhi, float Yh, float Yl, float bh,
                                           float Ybl, float beta, float rho, float c2f, float coef, bool raw,
                                           float zt, float r8, float r9, unsigned long long *bcol)
{
    const bool ends = !EC || rho < 0.9f;         // the margin guarantees Phi = 0 at the ends
    const float rho4 = 4.0f * rho;
    const float tb = (float)vlo - 0.5f;
    float d = Yh - tb;
    float d0 = d + bh;                           // Yh + bh - tb, exact on the 2^-10 grid
    float tc = tb - c2f;
    float s1p, mp, phip;
    if (vlo != vlo0 || !ends) boundary<EC>(d, Yl, d0, Ybl, tc, rho, rho4, s1p, mp, phip);
    else boundary<false>(d, Yl, d0, Ybl, tc, rho, rho4, s1p, mp, phip);
    float psip = mp + phip;                      // m(t) + Phi(t) of the row's top boundary
    auto weight = [&](float s1n, float phin) {
        float w = coef * (psip - phin);
        if (EXACT && !raw) {
            float mm = 0.5f * (fmaxf(0.0f, -s1p) + fminf(beta, -s1n));
            mm = fminf(fmaxf(mm, 0.0f), beta);
            const float zb = fmaf(-mm, r9, zt);
            w *= __builtin_amdgcn_rcpf(fmaf(zb, zb, r8));
        }
        return w;
    };
    unsigned long long *const last = bcol + vhi;
    for (unsigned long long *q = bcol + vlo; q < last; ++q) {
        d -= 1.0f;
        d0 -= 1.0f;
        tc += 1.0f;
        float s1n, mn, phin;
        boundary<EC>(d, Yl, d0, Ybl, tc, rho, rho4, s1n, mn, phin);
        lds_add_fixed(q, weight(s1n, phin));
        psip = mn + phin;
        s1p = s1n;
    }
    if (vlo <= vhi) {
        d -= 1.0f;
        d0 -= 1.0f;
        tc += 1.0f;
        float s1n = d + Yl, phin = 0.0f;
        if (vhi != vhi0 || !ends) {
            float mn;
            boundary<EC>(d, Yl, d0, Ybl, tc, rho, rho4, s1n, mn, phin);
        }
        lds_add_fixed(last, weight(s1n, phin));
    }
}

// Row weights of one TT voxel footprint, added to the band column bcol:
// rows [vlo, vhi] (clipped) of the unclipped range [vlo0, vhi0], which
// reaches beyond both ramps, so Phi is 0 at its first and last boundaries.
// Yh + Yl and Ybh + Ybl: middles of the rise and of the fall (high parts on
// the 2^-10 grid); eu, ed their half-widths.
__device__ __forceinline__ void sweep_rows_tt(int vlo0, int vhi0, int vlo, int vhi, float Yh, float Yl, float Ybh,
                                              float Ybl, float eu, float ed, float coef, unsigned long long *bcol)
{
    const float iu = __builtin_amdgcn_rcpf(fmaf(4.0f, eu, 1e-30f));
    const float id = __builtin_amdgcn_rcpf(fmaf(4.0f, ed, 1e-30f));
    const float tb = (float)vlo - 0.5f;
    float d = Yh - tb;
    float d0 = Ybh - tb;
    float s1, mp, phip;
    if (vlo != vlo0) boundary_tt<true>(d, Yl, d0, Ybl, eu, ed, iu, id, s1, mp, phip);
    else boundary_tt<false>(d, Yl, d0, Ybl, eu, ed, iu, id, s1, mp, phip);
    float psip = mp + phip;
    unsigned long long *const last = bcol + vhi;
    for (unsigned long long *q = bcol + vlo; q < last; ++q) {
        d -= 1.0f;
        d0 -= 1.0f;
        float mn, phin;
        boundary_tt<true>(d, Yl, d0, Ybl, eu, ed, iu, id, s1, mn, phin);
        lds_add_fixed(q, coef * (psip - phin));
        psip = mn + phin;
    }
    if (vlo <= vhi) {
        float phin = 0.0f;
        if (vhi != vhi0) {
            float mn;
            boundary_tt<true>(d - 1.0f, Yl, d0 - 1.0f, Ybl, eu, ed, iu, id, s1, mn, phin);
        }
        lds_add_fixed(last, coef * (psip - phin));
    }
}

// The TT footprint of a voxel whose top-face ramp has middle Yh + Yl: the
// half-widths |Y - c2| rho of its two faces; ramps that would overlap (a
// voxel shorter than its ramps) meet at the crossing of the sorted
// vertices, which moves each middle inwards by dl and narrows both ramps
// by dl.  Outputs the middles' low parts and the half-widths.
__device__ __forceinline__ void tt_ramps(float Yh, float Yl, float bl, float beta, float rho, float c2f,
                                         float &Ylu, float &Ybld, float &eu, float &ed)
{
    const float Yt = Yh + Yl;
    const float et = fabsf(Yt - c2f) * rho, eb = fabsf(Yt + beta - c2f) * rho;
    const float dl = 0.5f * fmaxf(et + eb - beta, 0.0f);
    Ylu = Yl - dl;
    Ybld = (Yl + bl) + dl;
    eu = et - dl;
    ed = eb - dl;
}

// The lanes of a record pass hold consecutive pieces of a column GW lanes
// apart, and the upper boundary u + 1/2 of piece s is the lower boundary of
// piece s + 1: each lane computes its lower prefix (also for s = n, the
// column's last boundary) and takes the upper one from lane + GW; the last
// slot of a pass computes its own.  column_prefix gets the same argument
// either way ((u + 1) - 1/2 = u + 1/2 exactly), so the records are unchanged.
__device__ __forceinline__ Mom shfl_mom(const Mom &m, int src)
{
    Mom r;
    r.a2 = __shfl(m.a2, src);
    r.sx = __shfl(m.sx, src);
    r.sy = __shfl(m.sy, src);
    r.sxx = __shfl(m.sxx, src);
    r.sxy = __shfl(m.sxy, src);
    r.syy = __shfl(m.syy, src);
    return r;
}

template <bool EXACT, bool EC, bool TT = false>
__device__ __forceinline__ void piece_pair_record(const DevGeom &G, const ViewGeom &V, const Column &C,
                                                  bool colok, int ufirst, int n, int s, bool last_slot,
                                                  int lane, int gw, float *rec)
{
    if constexpr (TT) {
        // footprints need no polygon moments
        if (colok && s < n) tt_record(G, V, C, ufirst + s, rec);
        return;
    }
    Mom lo = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (colok && s <= n) lo = column_prefix(G, V, C, (ufirst + s) - 0.5);
    Mom hi = shfl_mom(lo, lane + gw);
    if (colok && s < n) {
        if (last_slot) hi = column_prefix(G, V, C, (ufirst + s) + 0.5);
        piece_record<EXACT, EC>(G, V, C, ufirst + s, lo, hi, rec);
    }
}

// Record phase of the backprojection: LPV lanes l = (c, slot) compute the
// pieces of columns i0 + c of row j whose detector column u lies in
// [ulo, uhi], LPV / GW slots at a time.
template <bool EXACT, bool EC, int PMAX, int GW, int LPV, bool TT = false>
__device__ __forceinline__ void build_records(const DevGeom &G, const ViewGeom &V, int i0, int j,
                                              int ulo, int uhi, float *rec, int *npc, int l, int lane)
{
    constexpr int SLOTS = LPV / GW;
    const int c = l % GW;
    const int slot = l / GW;
    const int i = i0 + c;
    const bool colok = i < G.n1;
    Column C;
    int ufirst = 0, n = 0;
    if (colok) {
        C = make_column(G, V, i, j);
        ufirst = max((int)floor(C.chimin + 0.5), ulo);
        const int ulast = min((int)floor(C.chimax + 0.5), uhi);
        n = min(max(ulast - ufirst + 1, 0), PMAX);
    }
    if (slot == 0) npc[c] = n;
#pragma unroll
    for (int pass = 0; pass * SLOTS < PMAX; ++pass) {
        const int s = slot + pass * SLOTS;
        piece_pair_record<EXACT, EC, TT>(G, V, C, colok, ufirst, n, s, slot == SLOTS - 1, lane, GW,
                                         rec + (c * PMAX + min(s, PMAX - 1)) * kRecFloats);
    }
}

// A geometry's piece records, computed once: one thread per (view,
// column), its pieces in order (detector columns clipped to [0, M - 1], at
// most PMAX), the prefix moments of consecutive boundaries shared.  The
// arguments and operations are those of the kernels' own record stages
// (u + 1/2 = (u + 1) - 1/2 exactly, no contraction), so the records are the
// same bits and the kernels that read them give the same results.
template <int PMAX>
__global__ void __launch_bounds__(kBlock)
record_table_kernel(const DevGeom G, float *__restrict__ rec, int *__restrict__ cnt)
{
    const int64_t ncols = (int64_t)G.n1 * G.n2;
    const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= ncols * G.nviews) return;
    const int view = (int)(idx / ncols);
    const int rem = (int)(idx - (int64_t)view * ncols);
    const int j = rem / G.n1, i = rem - j * G.n1;
    const ViewGeom V = G.views[(size_t)view * G.vstride];
    const Column C = make_column(G, V, i, j);
    const int ufirst = max((int)floor(C.chimin + 0.5), 0);
    const int ulast = min((int)floor(C.chimax + 0.5), G.M - 1);
    const int n = min(max(ulast - ufirst + 1, 0), PMAX);
    cnt[idx] = n;
    float *out = rec + idx * PMAX * kRecFloats;
    Mom lo = column_prefix(G, V, C, ufirst - 0.5);
    for (int sl = 0; sl < n; ++sl) {
        const Mom hi = column_prefix(G, V, C, (ufirst + sl) + 0.5);
        float r[kRecFloats];
        piece_record<false, true>(G, V, C, ufirst + sl, lo, hi, r);
#pragma unroll
        for (int e = 0; e < kRecFloats; e += 4)
            *reinterpret_cast<float4 *>(out + sl * kRecFloats + e) = make_float4(r[e], r[e + 1], r[e + 2], r[e + 3]);
        lo = hi;
    }
}

// ------------------------------------------------------------ projection

// One work item of the projection: detector-column band item / nviews of view
// item % nviews.  smem holds the LDS layout described below.
template <bool EXACT, bool EC, int PMAX, bool TT = false, bool TAB = false>
__device__ __forceinline__ void project_item(const DevGeom &G, const int U, const int item,
                                             float *smem, const float *__restrict__ vol,
                                             float *__restrict__ proj, const unsigned *__restrict__ gmax)
{
    constexpr int GW = 16;
    const int view = item % G.nviews;
    const int u0 = (item / G.nviews) * U;
    const int ub = min(u0 + U, G.M) - 1;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const int Npad = G.N | 1;
    const int ngroups = (G.n1 + GW - 1) / GW;

    // one fixed-point band image [U][Npad] shared by the four waves, then the
    // row tables and a small reduction area
    unsigned long long *bins = reinterpret_cast<unsigned long long *>(smem);
    int *rowStart = reinterpret_cast<int *>(bins + U * Npad);
    int *rowQ = rowStart + (G.n2 + 1);
    int *part = rowQ + G.n2;
    unsigned *red = reinterpret_cast<unsigned *>(part + kBlock);

    for (int idx = tid; idx < U * Npad; idx += kBlock) bins[idx] = 0ull;

    const ViewGeom V = G.views[(size_t)view * G.vstride];

    // Column groups of each row j meeting the band's wedge: the chi1 range of
    // a group's base rectangle (extremes at its corners) must meet
    // [u0 - 1/2, ub + 1/2].  chi1 is monotone in x1, so the hits are
    // contiguous in the group index.  FP32 with a margin is conservative.
    {
        const float fb = (float)V.fb1;
        const float e1x = (float)V.e1x, e1y = (float)V.e1y, dx = (float)V.dx, dy = (float)V.dy;
        const float lo_t = u0 - 0.5f - 0.02f, hi_t = ub + 0.5f + 0.02f;
        const int rows_per = (G.n2 + kBlock - 1) / kBlock;
        int local = 0;
        for (int r = 0; r < rows_per; ++r) {
            const int j = tid * rows_per + r;
            if (j >= G.n2) break;
            const float y0 = (float)(G.x2lo + j * G.a2 - V.s2), y1 = y0 + (float)G.a2;
            int qa = -1, qb = -2;
            for (int q = 0; q < ngroups; ++q) {
                const float x0 = (float)(G.x1lo + q * GW * G.a1 - V.s1);
                const float x1 = (float)(G.x1lo + min((q + 1) * GW, G.n1) * G.a1 - V.s1);
                float mn = 1e30f, mx = -1e30f;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const float px = (k & 1) ? x1 : x0, py = (k & 2) ? y1 : y0;
                    const float ch = (float)V.c1 + fb * (e1x * px + e1y * py) / (dx * px + dy * py);
                    mn = fminf(mn, ch);
                    mx = fmaxf(mx, ch);
                }
                if (mx >= lo_t && mn <= hi_t) {
                    if (qa < 0) qa = q;
                    qb = q;
                }
            }
            rowQ[j] = qa;
            const int cnt = qa >= 0 ? qb - qa + 1 : 0;
            rowStart[j] = cnt;   // counts for now
            local += cnt;
        }
        part[tid] = local;
        __syncthreads();
        if (tid == 0) {
            int acc = 0;
            for (int t = 0; t < kBlock; ++t) {
                const int v = part[t];
                part[t] = acc;
                acc += v;
            }
            rowStart[G.n2] = acc;
        }
        __syncthreads();
        int acc = part[tid];
        for (int r = 0; r < rows_per; ++r) {
            const int j = tid * rows_per + r;
            if (j >= G.n2) break;
            const int cnt = rowStart[j];
            rowStart[j] = acc;
            acc += cnt;
        }
        __syncthreads();
    }
    const int total = rowStart[G.n2];

    const float c2f = (float)V.c2;
    const float a3f = (float)G.a3;
    const float zt0 = (float)(G.x3lo + G.a3 - V.s3);   // x3 of the top of voxel 0, minus s3
    const bool raw = G.raw_volume != 0;
    const bool vec_rows = (G.n1 & 3) == 0 && (reinterpret_cast<uintptr_t>(vol) & 15) == 0;

    // Group gi of the wedge -> (row j, first column i0).
    auto group = [&](int gi, int &j, int &i0) {
        int lo = 0, hi = G.n2;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (rowStart[mid] <= gi) lo = mid; else hi = mid;
        }
        j = lo;
        i0 = (rowQ[j] + (gi - rowStart[j])) * GW;
    };
    // mu of columns i0 .. i0+15 of row j at slice k (clamped; zero past n1)
    auto load_mu = [&](int j, int i0, int k, bool full, float mu[GW]) {
        const float *rowp = vol + ((size_t)min(k, G.n3 - 1) * G.n2 + j) * G.n1 + i0;
        if (full) {
#pragma unroll
            for (int q = 0; q < GW / 4; ++q) {
                const float4 t4 = reinterpret_cast<const float4 *>(rowp)[q];
                mu[4 * q] = t4.x; mu[4 * q + 1] = t4.y; mu[4 * q + 2] = t4.z; mu[4 * q + 3] = t4.w;
            }
        } else {
#pragma unroll
            for (int c = 0; c < GW; ++c) mu[c] = (i0 + c < G.n1) ? rowp[c] : 0.0f;
        }
    };

    // Scale of the fixed-point image from the largest |mu| in the wedge (as
    // the bit pattern of |mu|, so Inf and NaN compare above every finite
    // value): times a geometric bound on one weight it must stay below 2^51
    // (each contribution converts exactly, see lds_add_fixed), times a bound
    // on a pixel's weight sum below 2^61 (the 64-bit sums cannot overflow).
    // The second bound is the binding one, so a contribution is kept to
    // about 2^-55 of the largest possible pixel sum of the band.  With gmax
    // (the per-group maxima of group_max_kernel) the wedge maximum is a
    // lookup per group; without it the wedge is read once more here.
    unsigned mxl = 0u;
    if (gmax) {
        for (int gi = tid; gi < total; gi += kBlock) {
            int j, i0;
            group(gi, j, i0);
            mxl = max(mxl, gmax[j * ngroups + i0 / GW]);
        }
    } else {
        for (int gi = wave; gi < total; gi += kWaves) {
            int j, i0;
            group(gi, j, i0);
            const bool full = vec_rows && (i0 + GW <= G.n1);
            for (int kc = 0; kc < G.n3; kc += kWave) {
                float mu[GW];
                load_mu(j, i0, kc + lane, full, mu);
                if (kc + lane < G.n3) {
#pragma unroll
                    for (int c = 0; c < GW; ++c) mxl = max(mxl, __float_as_uint(mu[c]) & 0x7fffffffu);
                }
            }
        }
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) mxl = max(mxl, (unsigned)__shfl_xor((int)mxl, off));
    if (lane == 0) red[wave] = mxl;
    __syncthreads();
    const unsigned mxb = max(max(red[0], red[1]), max(red[2], red[3]));
    const bool finite = mxb < 0x7f800000u;
    int sc = 0;
    if (finite && mxb != 0u) {
        int e1, e2;
        frexp((double)__uint_as_float(mxb) * (raw ? G.wone_bound_raw : G.wone_bound), &e1);
        frexp((double)__uint_as_float(mxb) * (raw ? G.wsum_bound_raw : G.wsum_bound), &e2);
        sc = min(51 - e1, 61 - e2);
    }
    const int ngi = (finite && mxb != 0u) ? total : 0;   // all-zero wedge: nothing to add

    for (int gi = wave; gi < ngi; gi += kWaves) {
        int j, i0;
        group(gi, j, i0);

        // Piece records stay in the registers of the lanes that computed them
        // (lane c + 16 s holds slot s of column c, pass q in rq[q]); the voxel
        // loop fetches them with readlane, so no LDS read (and no wait on the
        // outstanding LDS atomics) sits between consecutive pieces.
        constexpr int PASSES = PMAX / 4;
        float rq[PASSES][kRecFloats];
        int ncol = 0;
        if constexpr (TAB) {
            // the geometry's records: the column's pieces that fall in the band
            const int c = lane & 15, slot = lane >> 4;
            const int i = i0 + c;
            if (i < G.n1) {
                const size_t col = ((size_t)view * G.vstride * G.n2 + j) * G.n1 + i;
                const int nt = G.rtab_n[col];
                const float *rc = G.rtab + col * G.rtab_pmax * kRecFloats;
                const int uf = nt > 0 ? __float_as_int(rc[0]) : 0;
                const int off = max(u0 - uf, 0);
                ncol = min(max(min(nt, ub - uf + 1) - off, 0), PMAX);
#pragma unroll
                for (int q = 0; q < PASSES; ++q) {
                    const int sl = slot + 4 * q;
                    if (sl < ncol) {
                        const float4 *r4 = reinterpret_cast<const float4 *>(rc + (off + sl) * kRecFloats);
#pragma unroll
                        for (int e = 0; e < kRecFloats / 4; ++e) {
                            const float4 t4 = r4[e];
                            rq[q][4 * e] = t4.x; rq[q][4 * e + 1] = t4.y; rq[q][4 * e + 2] = t4.z; rq[q][4 * e + 3] = t4.w;
                        }
                    }
                }
            }
        } else {
            const int c = lane & 15, slot = lane >> 4;
            const int i = i0 + c;
            const bool colok = i < G.n1;
            Column C;
            int ufirst = 0;
            if (colok) {
                C = make_column(G, V, i, j);
                ufirst = max((int)floor(C.chimin + 0.5), u0);
                const int ulast = min((int)floor(C.chimax + 0.5), ub);
                ncol = min(max(ulast - ufirst + 1, 0), PMAX);
            }
#pragma unroll
            for (int q = 0; q < PASSES; ++q)
                piece_pair_record<EXACT, EC, TT>(G, V, C, colok, ufirst, ncol, slot + 4 * q, slot == 3, lane, 16,
                                                 rq[q]);
        }
        if (__ballot(ncol > 0) == 0) continue;
        const bool full = vec_rows && (i0 + GW <= G.n1);

        // With cached records each lane takes KP slices (k and k + 64): one
        // broadcast of a piece record then serves 64 KP voxels.
        constexpr int KP = TAB ? 2 : 1;
        for (int kc = 0; kc < G.n3; kc += kWave * KP) {
            float mu[KP][GW];
            float kf[KP], zt[KP], zc[KP];
            bool kv[KP];
#pragma unroll
            for (int h = 0; h < KP; ++h) {
                const int k = kc + h * kWave + lane;
                kv[h] = k < G.n3;
                load_mu(j, i0, k, full, mu[h]);
                kf[h] = (float)k;
                zt[h] = fmaf(kf[h], a3f, zt0);        // top of voxel k, relative to s3
                zc[h] = zt[h] - 0.5f * a3f;           // centre of voxel k
            }
#pragma unroll
            for (int c = 0; c < GW; ++c) {
                const int np = __builtin_amdgcn_readlane(ncol, c);
                if (np == 0) continue;
                float base[KP];
                bool any = false;
#pragma unroll
                for (int h = 0; h < KP; ++h) {
                    base[h] = kv[h] ? mu[h][c] : 0.0f;
                    any = any || base[h] != 0.0f;
                }
                if (__ballot(any) == 0) continue;
                const float r8c = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(rq[0][8]), c));
#pragma unroll
                for (int h = 0; h < KP; ++h) {
                    if (TT)   // the central ray's |r| (its min(a1/|r1|, a2/|r2|) is in the records)
                        base[h] = base[h] * sqrtf(fmaf(zc[h], zc[h], r8c));
                    else if (!EXACT && !raw)
                        base[h] = base[h] * __builtin_amdgcn_rcpf(fmaf(zc[h], zc[h], r8c));
                    base[h] = ldexpf(base[h], sc);
                }
                for (int p = 0; p < np; ++p) {
                    const int src = c + 16 * (p & 3);
                    float r[kRecFloats];
                    if (PASSES == 1 || p < 4) {
#pragma unroll
                        for (int e = 0; e < kRecFloats; ++e)
                            r[e] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(rq[0][e]), src));
                    } else {
#pragma unroll
                        for (int e = 0; e < kRecFloats; ++e)
                            r[e] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(rq[PASSES - 1][e]), src));
                    }
                    const int u = __float_as_int(r[0]);
                    const float beta = r[6], rho = r[7];
                    unsigned long long *bcol = bins + (u - u0) * Npad;
#pragma unroll
                    for (int h = 0; h < KP; ++h) {
                        const float coef = base[h] * r[1];
                        const float Yh = fmaf(-kf[h], r[4], r[2]);
                        const float Yl = fmaf(-kf[h], r[5], r[3]);
                        int vlo0, vhi0;
                        row_range_unclipped<EC>(Yh + Yl, beta, r[10], c2f, vlo0, vhi0);
                        if constexpr (TT) {
                            float Ylu, Ybld, eu, ed;
                            tt_ramps(Yh, Yl, r[5], beta, rho, c2f, Ylu, Ybld, eu, ed);
                            sweep_rows_tt(vlo0, vhi0, max(vlo0, 0), min(vhi0, G.N - 1), Yh, Ylu, Yh + r[4], Ybld,
                                          eu, ed, coef, bcol);
                        } else {
                            // bottom face Y(k - 1): high part Yh + bh (exact on the 2^-10 grid), low part Yl + bl
                            sweep_rows<EC, EXACT>(vlo0, vhi0, max(vlo0, 0), min(vhi0, G.N - 1), Yh, Yl, r[4],
                                                  Yl + r[5], beta, rho, c2f, coef, raw, zt[h], r[11], r[9], bcol);
                        }
                    }
                }
            }
        }
    }
    __syncthreads();

    // Coalesced flush of the band: S = sum * 2^-s, times the pixel factor
    // (second phase).  A non-finite input in the wedge makes the band NaN.
    const int Ub = ub - u0 + 1;
    for (int idx = tid; idx < Ub * G.N; idx += kBlock) {
        const int du = idx % Ub, v = idx / Ub;
        const int u = u0 + du;
        float s = finite ? (float)ldexp(fixed_to_double(bins[du * Npad + v]), -sc) : __builtin_nanf("");
        if (G.sigma) s *= G.sigma[((size_t)view * G.vstride * G.sigma_views * G.N + v) * G.M + u];
        proj[((size_t)view * G.vstride * G.N + v) * G.M + u] = s;
    }
}

// Register budgets: the projection is held to 96 VGPRs (5 waves per SIMD,
// spills outside the voxel loop) and the backprojection to 168 (3 waves per
// SIMD); both ran about 20% faster at 512^3 x 248 views than at their
// natural 190-220 VGPRs with 2 waves per SIMD, and the projection 3% faster
// at 5 waves than at 4.
template <bool EXACT, bool EC, int PMAX, bool TT = false, bool TAB = false>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(5)))
project_kernel(const DevGeom G, const int U, const int nbands, const float *__restrict__ vol,
               float *__restrict__ proj, const unsigned *__restrict__ gmax, const double *__restrict__ stop)
{
    extern __shared__ __align__(16) float smem[];
    if (stop && *stop != 0.0) return;   // a converged solver: nothing to do
    // Workgroups go to the 8 XCDs round robin.  XCD x takes bands x, x + 8,
    // x + 16, ..., each for all views in order: the costly central bands are
    // spread over all XCDs, and the workgroups an XCD runs at a time share a
    // band and neighbouring views, so their wedges overlap in its L2.
    const int slot = blockIdx.x >> 3;
    const int band = (blockIdx.x & 7) + 8 * (slot / G.nviews);
    if (band >= nbands) return;
    project_item<EXACT, EC, PMAX, TT, TAB>(G, U, band * G.nviews + slot % G.nviews, smem, vol, proj, gmax);
}

// gmax[j * ngroups + q] = the largest |mu| bit pattern over the columns
// 16 q .. 16 q + 15 (< n1) of row j and all slices: one wave per (j, q),
// lanes over k.  The projection's wedge maxima are then lookups.
__global__ void __launch_bounds__(kBlock)
group_max_kernel(const DevGeom G, const float *__restrict__ vol, unsigned *__restrict__ gmax,
                 const double *__restrict__ stop)
{
    if (stop && *stop != 0.0) return;
    constexpr int GW = 16;
    const int ngroups = (G.n1 + GW - 1) / GW;
    const int cell = blockIdx.x * kWaves + threadIdx.x / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    if (cell >= G.n2 * ngroups) return;
    const int j = cell / ngroups, i0 = (cell % ngroups) * GW;
    const bool full = (G.n1 & 3) == 0 && (reinterpret_cast<uintptr_t>(vol) & 15) == 0 && i0 + GW <= G.n1;
    unsigned mxl = 0u;
    for (int k = lane; k < G.n3; k += kWave) {
        const float *rowp = vol + ((size_t)k * G.n2 + j) * G.n1 + i0;
        if (full) {
#pragma unroll
            for (int q = 0; q < GW / 4; ++q) {
                const float4 t4 = reinterpret_cast<const float4 *>(rowp)[q];
                mxl = max(mxl, max(max(__float_as_uint(t4.x) & 0x7fffffffu, __float_as_uint(t4.y) & 0x7fffffffu),
                                   max(__float_as_uint(t4.z) & 0x7fffffffu, __float_as_uint(t4.w) & 0x7fffffffu)));
            }
        } else {
            for (int c = 0; c < GW && i0 + c < G.n1; ++c) mxl = max(mxl, __float_as_uint(rowp[c]) & 0x7fffffffu);
        }
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) mxl = max(mxl, (unsigned)__shfl_xor((int)mxl, off));
    if (lane == 0) gmax[cell] = mxl;
}

// ------------------------------------------------------------ backprojection

// One work item of the backprojection: a stack of GW columns x 64 kp voxels
// (kp = 1 or 2), gathered in kp 64-voxel passes that share each view's piece
// records and detector window (with kp = 2, half their cost per voxel).
template <bool EXACT, bool EC, int PMAX, int GW, bool TT = false, bool TAB = false>
__device__ __forceinline__ void backproject_item(const DevGeom &G, const int ngroups,
                                                 const int nkchunks, const int kp, const int winCap,
                                                 const int item, float *smem,
                                                 const float *__restrict__ proj,
                                                 float *__restrict__ vol)
{
    const int kch = item % nkchunks;
    const int t = item / nkchunks;
    const int q = t % ngroups;
    const int j = t / ngroups;
    constexpr int KP = kBackPasses;
    const int i0 = q * GW;
    const int k0 = kch * kWave * kp;
    const int tid = threadIdx.x, lane = tid & (kWave - 1);
    const int wave = TAB ? __builtin_amdgcn_readfirstlane(tid / kWave) : tid / kWave;
    const int kmax = min(k0 + kWave * kp, G.n3) - 1;

    // One record pass covers RV of the wave's views (w, w + 4, ...): LPV
    // lanes per view, so narrow stacks do not leave most lanes idle in the
    // FP64 stage.  Per view: records, piece counts, window bounds.
    constexpr int LPV = GW * (PMAX < kWave / GW ? PMAX : kWave / GW);
    constexpr int RV = kWave / LPV;
    constexpr int recView = back_rec_floats(GW, PMAX);
    const int recFloats = RV * recView;
    const int waveFloats = ((recFloats + winCap + 3) / 4) * 4;
    float *rec = smem + wave * waveFloats;
    float *win = rec + recFloats;

    const float a3f = (float)G.a3;
    const bool raw = G.raw_volume != 0;

    float acc[KP][GW];
#pragma unroll
    for (int ps = 0; ps < KP; ++ps)
#pragma unroll
        for (int c = 0; c < GW; ++c) acc[ps][c] = 0.0f;

    for (int vb = wave; vb < G.nviews; vb += kWaves * RV) {
        if constexpr (TAB) {
            // the geometry's records of the stack, view by view, into LDS
#pragma unroll
            for (int r = 0; r < RV; ++r) {
                const int view = vb + r * kWaves;
                if (view >= G.nviews) break;
                float *rv = rec + r * recView;
                int *npv = reinterpret_cast<int *>(rv + GW * PMAX * kRecFloats);
                const size_t col0 = ((size_t)view * G.vstride * G.n2 + j) * G.n1 + i0;
                const int ncv = min(GW, G.n1 - i0);
                const int tp = G.rtab_pmax;
                const float4 *src = reinterpret_cast<const float4 *>(G.rtab + col0 * tp * kRecFloats);
                if (tp == PMAX) {
                    // one contiguous block
                    for (int q4 = lane; q4 < ncv * PMAX * kRecFloats / 4; q4 += kWave)
                        reinterpret_cast<float4 *>(rv)[q4] = src[q4];
                } else {
                    // a table of tp <= PMAX slots per column (batched launches keep PMAX = 8)
                    constexpr int F4 = kRecFloats / 4;
                    for (int q4 = lane; q4 < ncv * tp * F4; q4 += kWave) {
                        const int cs = q4 / F4, c = cs / tp, sl = cs - c * tp;
                        reinterpret_cast<float4 *>(rv)[(c * PMAX + sl) * F4 + (q4 - cs * F4)] = src[q4];
                    }
                }
                if (lane < GW) npv[lane] = lane < ncv ? G.rtab_n[col0 + lane] : 0;
            }
        } else {
            // The accumulators wait in the (idle) window area while the FP64
            // record stage, the kernel's register peak, runs.
#pragma unroll
            for (int ps = 0; ps < KP; ++ps)
#pragma unroll
                for (int c = 0; c < GW; ++c) win[(ps * GW + c) * kWave + lane] = acc[ps][c];
            wave_sync();
            const int r = lane / LPV;
            const int view = vb + r * kWaves;
            float *rv = rec + r * recView;
            if (view < G.nviews)
                build_records<EXACT, EC, PMAX, GW, LPV, TT>(G, G.views[(size_t)view * G.vstride], i0, j, 0, G.M - 1, rv,
                                                        reinterpret_cast<int *>(rv + GW * PMAX * kRecFloats),
                                                        lane % LPV, lane);
        }
        wave_sync();

        // detector window of the stack per view: columns of all pieces, rows
        // of the chunk's top voxel (smallest chi2) to its bottom voxel (the
        // first view's in registers, the others' after their piece counts)
        int wb0[4];
#pragma unroll
        for (int r = 0; r < RV; ++r) {
            if (vb + r * kWaves >= G.nviews) break;
            const float *rv = rec + r * recView;
            int *npv = reinterpret_cast<int *>(const_cast<float *>(rv) + GW * PMAX * kRecFloats);
            const float c2f = (float)G.views[(size_t)(vb + r * kWaves) * G.vstride].c2;
            int wu0 = 1 << 30, wu1 = -1, wv0 = 1 << 30, wv1 = -1;
            const int c = lane % GW, s0 = lane / GW;
            for (int s = s0; s < PMAX; s += kWave / GW) {
                if (s < npv[c]) {
                    const float *r = rv + (c * PMAX + s) * kRecFloats;
                    const int u = __float_as_int(r[0]);
                    const float beta = r[6], mfac = r[10];
                    const float Ytop_hi = fmaf(-(float)kmax, r[4], r[2]) + fmaf(-(float)kmax, r[5], r[3]);
                    const float Ytop_lo = fmaf(-(float)k0, r[4], r[2]) + fmaf(-(float)k0, r[5], r[3]);
                    int a, b, a2, b2;
                    row_range<EC>(Ytop_hi, beta, mfac, c2f, G.N, a, b);
                    row_range<EC>(Ytop_lo, beta, mfac, c2f, G.N, a2, b2);
                    wu0 = min(wu0, u); wu1 = max(wu1, u);
                    wv0 = min(wv0, min(a, a2)); wv1 = max(wv1, max(b, b2));
                }
            }
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                wu0 = min(wu0, __shfl_xor(wu0, off));
                wu1 = max(wu1, __shfl_xor(wu1, off));
                wv0 = min(wv0, __shfl_xor(wv0, off));
                wv1 = max(wv1, __shfl_xor(wv1, off));
            }
            if (r == 0) {
                wb0[0] = wu0; wb0[1] = wu1; wb0[2] = wv0; wb0[3] = wv1;
            } else if (lane == 0) {
                npv[GW] = wu0; npv[GW + 1] = wu1; npv[GW + 2] = wv0; npv[GW + 3] = wv1;
            }
        }
        if constexpr (!TAB) {
#pragma unroll
            for (int ps = 0; ps < KP; ++ps)
#pragma unroll
                for (int c = 0; c < GW; ++c) acc[ps][c] = win[(ps * GW + c) * kWave + lane];
        }
        wave_sync();

#pragma unroll 1
        for (int r = 0; r < RV; ++r) {
        const int view = vb + r * kWaves;
        if (view >= G.nviews) break;
        const ViewGeom V = G.views[(size_t)view * G.vstride];
        const float c2f = (float)V.c2;
        const float *sgv = G.sigma ? G.sigma + (size_t)view * G.vstride * G.sigma_views * G.N * G.M : nullptr;
        const float *recv = rec + r * recView;
        const int *npc = reinterpret_cast<const int *>(recv + GW * PMAX * kRecFloats);
        int wu0 = wb0[0], wu1 = wb0[1], wv0 = wb0[2], wv1 = wb0[3];
        if (r > 0) {
            wu0 = npc[GW]; wu1 = npc[GW + 1]; wv0 = npc[GW + 2]; wv1 = npc[GW + 3];
        }
        if constexpr (TAB) {
            // the window bounds are the same in every lane
            wu0 = __builtin_amdgcn_readfirstlane(wu0);
            wu1 = __builtin_amdgcn_readfirstlane(wu1);
            wv0 = __builtin_amdgcn_readfirstlane(wv0);
            wv1 = __builtin_amdgcn_readfirstlane(wv1);
        }
        if (wu1 < wu0 || wv1 < wv0) continue;
        // one spare row each side absorbs FP32 rounding of intermediate k
        wv0 = max(wv0 - 1, 0);
        wv1 = min(wv1 + 1, G.N - 1);
        const int Wd = wu1 - wu0 + 1;
        const int H = wv1 - wv0 + 1;
        const int Hp = H | 1;
        const float *pv = proj + (size_t)view * G.vstride * G.N * G.M;

        const bool useWin = Wd * Hp <= winCap;
        if (useWin) {
            for (int idx = lane; idx < Wd * H; idx += kWave) {
                const int uu = idx % Wd, vv = idx / Wd;
                const size_t off = (size_t)(wv0 + vv) * G.M + (wu0 + uu);
                float val = pv[off];
                if (sgv) val *= sgv[off];
                win[uu * Hp + vv] = val;
            }
        }
        wave_sync();

        // the gather, with the window read from LDS (WIN) or global memory.
        // piece(): the row sum of one piece for one voxel (lanes over k),
        // times the piece's coefficient by the caller.
        auto gather = [&](auto winTag, auto npTag) {
        constexpr bool WIN = decltype(winTag)::value;
        constexpr int NP = decltype(npTag)::value;   // passes (a bound for the second form)
        auto piece = [&](const float4 &r0, const float4 &r1, const float4 &r2, const int u, const float *wcol,
                         const float kf, const float zt, const bool kv) -> float {
            const float Yh = fmaf(-kf, r1.x, r0.z);
            const float Yl = fmaf(-kf, r1.y, r0.w);
            const float Ybh = Yh + r1.x, Ybl = Yl + r1.y;   // bottom face Y(k - 1), exact high part
            const float beta = r1.z, rho = r1.w, rho4 = 4.0f * r1.w;
            // rows clipped to the detector and the window; as in the
            // projection, Phi at the first and last boundaries of the
            // unclipped range is exactly 0
            int vlo0, vhi0;
            row_range_unclipped<EC>(Yh + Yl, beta, r2.z, c2f, vlo0, vhi0);
            const bool ends = !EC || rho < 0.9f;
            const int vlo = max(max(vlo0, 0), wv0);
            const int vhi = kv ? min(min(vhi0, G.N - 1), wv1) : vlo - 1;
            if constexpr (TT) {
                // the TT axial footprint's row integrals (Phi is exactly 0
                // at the ends of the unclipped range, computed or not)
                float Ylu, Ybld, eu, ed;
                tt_ramps(Yh, Yl, r1.y, beta, rho, c2f, Ylu, Ybld, eu, ed);
                const float iu = __builtin_amdgcn_rcpf(fmaf(4.0f, eu, 1e-30f));
                const float id = __builtin_amdgcn_rcpf(fmaf(4.0f, ed, 1e-30f));
                const float tb = (float)vlo - 0.5f;
                float d = Yh - tb, d0 = Ybh - tb;
                float s1, mp, phip;
                boundary_tt<true>(d, Ylu, d0, Ybld, eu, ed, iu, id, s1, mp, phip);
                float psip = mp + phip, ap = 0.0f;
                for (int v = vlo; v <= vhi; ++v) {
                    d -= 1.0f;
                    d0 -= 1.0f;
                    float mn, phin;
                    boundary_tt<true>(d, Ylu, d0, Ybld, eu, ed, iu, id, s1, mn, phin);
                    const float val = WIN ? wcol[v] : pv[(size_t)v * G.M + u];
                    ap = fmaf(psip - phin, val, ap);
                    psip = mn + phin;
                }
                return ap;
            }
            // boundaries as in sweep_rows; row weight m(t) + Phi(t) - Phi(t + 1)
            const float tb = (float)vlo - 0.5f;
            float d = Yh - tb;
            float d0 = d + r1.x;                     // Ybh - tb, exact on the 2^-10 grid
            float tc = tb - c2f;
            float s1p, mp, phip;
            if (vlo != vlo0 || !ends) boundary<EC>(d, Yl, d0, Ybl, tc, rho, rho4, s1p, mp, phip);
            else boundary<false>(d, Yl, d0, Ybl, tc, rho, rho4, s1p, mp, phip);
            float psip = mp + phip;
            float ap = 0.0f;          // sum of row weight [1/r^2] val_v
            auto row = [&](float val) {
                d -= 1.0f;
                d0 -= 1.0f;
                tc += 1.0f;
                float s1n, mn, phin;
                boundary<EC>(d, Yl, d0, Ybl, tc, rho, rho4, s1n, mn, phin);
                float w = psip - phin;
                if (EXACT && !raw) {
                    float mm = 0.5f * (fmaxf(0.0f, -s1p) + fminf(beta, -s1n));
                    mm = fminf(fmaxf(mm, 0.0f), beta);
                    const float zb = fmaf(-mm, r2.y, zt);
                    w *= __builtin_amdgcn_rcpf(fmaf(zb, zb, r2.w));
                }
                ap = fmaf(w, val, ap);
                psip = mn + phin;
                s1p = s1n;
            };
            if (WIN) {
                const float *const last = wcol + vhi;
                for (const float *q = wcol + vlo; q < last; ++q) row(*q);
                if (vlo <= vhi) {
                    // last row: Phi at the last boundary of the unclipped
                    // range is exactly 0
                    d -= 1.0f;
                    d0 -= 1.0f;
                    tc += 1.0f;
                    float s1n = d + Yl, phin = 0.0f;
                    if (vhi != vhi0 || !ends) {
                        float mn;
                        boundary<EC>(d, Yl, d0, Ybl, tc, rho, rho4, s1n, mn, phin);
                    }
                    float w = psip - phin;
                    if (EXACT && !raw) {
                        float mm = 0.5f * (fmaxf(0.0f, -s1p) + fminf(beta, -s1n));
                        mm = fminf(fmaxf(mm, 0.0f), beta);
                        const float zb = fmaf(-mm, r2.y, zt);
                        w *= __builtin_amdgcn_rcpf(fmaf(zb, zb, r2.w));
                    }
                    ap = fmaf(w, *last, ap);
                }
            } else {
                for (int v = vlo; v <= vhi; ++v) {
                    const size_t off = (size_t)v * G.M + u;
                    float val = pv[off];
                    if (sgv) val *= sgv[off];
                    row(val);
                }
            }
            return ap;
        };
        auto record = [&](const float *rc, int p, float4 &r0, float4 &r1, float4 &r2) {
            r0 = *reinterpret_cast<const float4 *>(rc + p * kRecFloats);
            r1 = *reinterpret_cast<const float4 *>(rc + p * kRecFloats + 4);
            r2 = *reinterpret_cast<const float4 *>(rc + p * kRecFloats + 8);
        };
        auto base_of = [&](const float *rc, float kf) {
            const float zc = fmaf(kf, a3f, (float)(G.x3lo + G.a3 - V.s3)) - 0.5f * a3f;
            float base = 1.0f;
            if (TT) base = sqrtf(fmaf(zc, zc, rc[8]));
            else if (!EXACT && !raw) base = __builtin_amdgcn_rcpf(fmaf(zc, zc, rc[8]));
            return base;
        };
        if constexpr (TAB && NP > 1) {
            // Each piece record is read once and serves the NP passes; the
            // piece count, u and the window bounds are the same in every
            // lane (scalar registers).  A voxel's pieces are summed in piece
            // order, as below.  (With one pass the per-lane form below is
            // faster.)
            bool live[NP], kv[NP];
            float kf[NP], zt[NP];
#pragma unroll
            for (int ps = 0; ps < NP; ++ps) {
                live[ps] = k0 + ps * kWave < G.n3;   // uniform
                const int k = k0 + ps * kWave + lane;
                kv[ps] = k < G.n3;
                kf[ps] = (float)k;
                zt[ps] = fmaf(kf[ps], a3f, (float)(G.x3lo + G.a3 - V.s3));
            }
#pragma unroll
            for (int c = 0; c < GW; ++c) {
                const int np = __builtin_amdgcn_readfirstlane(npc[c]);
                if (np == 0) continue;
                const float *rc = recv + c * PMAX * kRecFloats;
                float base[NP], a[NP];
#pragma unroll
                for (int ps = 0; ps < NP; ++ps) {
                    base[ps] = base_of(rc, kf[ps]);
                    a[ps] = 0.0f;
                }
                for (int p = 0; p < np; ++p) {
                    float4 r0, r1, r2;
                    record(rc, p, r0, r1, r2);
                    const int u = __builtin_amdgcn_readfirstlane(__float_as_int(r0.x));
                    const float *wcol = win + (u - wu0) * Hp - wv0;
#pragma unroll
                    for (int ps = 0; ps < NP; ++ps)
                        if (live[ps])
                            a[ps] = fmaf(base[ps] * r0.y, piece(r0, r1, r2, u, wcol, kf[ps], zt[ps], kv[ps]), a[ps]);
                }
#pragma unroll
                for (int ps = 0; ps < NP; ++ps)
                    if (live[ps]) acc[ps][c] += a[ps];
            }
        } else {
#pragma unroll
            for (int ps = 0; ps < NP; ++ps) {
                if (ps >= kp || k0 + ps * kWave >= G.n3) break;   // unused pass
                const int k = k0 + ps * kWave + lane;
                const bool kv = k < G.n3;
                const float kf = (float)k;
                const float zt = fmaf(kf, a3f, (float)(G.x3lo + G.a3 - V.s3));
#pragma unroll
                for (int c = 0; c < GW; ++c) {
                    const int np = npc[c];
                    if (np == 0) continue;
                    const float *rc = recv + c * PMAX * kRecFloats;
                    const float base = base_of(rc, kf);
                    float a = 0.0f;
                    for (int p = 0; p < np; ++p) {
                        float4 r0, r1, r2;
                        record(rc, p, r0, r1, r2);
                        const int u = __float_as_int(r0.x);
                        a = fmaf(base * r0.y, piece(r0, r1, r2, u, win + (u - wu0) * Hp - wv0, kf, zt, kv), a);
                    }
                    acc[ps][c] += a;
                }
            }
        }
        };
        using P1 = std::integral_constant<int, 1>;
        using P2 = std::integral_constant<int, KP>;
        if (TAB && kp == 1) {
            if (useWin) gather(std::true_type{}, P1{});
            else gather(std::false_type{}, P1{});
        } else {
            if (useWin) gather(std::true_type{}, P2{});
            else gather(std::false_type{}, P2{});
        }
        wave_sync();
        }
    }

    // Sum the four waves' partial sums in a fixed order; one store per voxel.
    float *red = smem;   // [kWaves][GW][kWave], aliases the per-wave areas
#pragma unroll
    for (int ps = 0; ps < KP; ++ps) {
        if (ps >= kp) break;
        __syncthreads();
#pragma unroll
        for (int c = 0; c < GW; ++c) red[(wave * GW + c) * kWave + lane] = acc[ps][c];
        __syncthreads();
        const int k = k0 + ps * kWave + lane;
        for (int c = wave; c < GW; c += kWaves) {
            const int i = i0 + c;
            float s = red[(0 * GW + c) * kWave + lane];
#pragma unroll
            for (int w = 1; w < kWaves; ++w) s += red[(w * GW + c) * kWave + lane];
            if (k < G.n3 && i < G.n1) vol[((size_t)k * G.n2 + j) * G.n1 + i] = s;
        }
    }
}

template <bool EXACT, bool EC, int PMAX, int GW, bool TT = false, bool TAB = false>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3)))
backproject_kernel(const DevGeom G, const int ngroups, const int nkchunks, const int kp, const int items,
                   const int chunk, const int winCap, const float *__restrict__ proj,
                   float *__restrict__ vol, const double *__restrict__ stop)
{
    extern __shared__ __align__(16) float smem[];
    if (stop && *stop != 0.0) return;
    const int item = (blockIdx.x & 7) * chunk + (blockIdx.x >> 3);
    if (item >= items) return;
    backproject_item<EXACT, EC, PMAX, GW, TT, TAB>(G, ngroups, nkchunks, kp, winCap, item, smem, proj, vol);
}

// The backprojection with one detector window per workgroup (cached records
// only): the four waves take the same view at a time, wave w the columns
// w GW/4 .. (w + 1) GW/4 - 1 of the stack, so the window (staged by all 256
// threads) can be four times as large as a wave's own -- for detectors whose
// pixels are small against the voxels, where a wave's window does not fit
// LDS.  Each wave keeps one partial sum per view class (view mod 4), summed
// in view order and combined as ((c0 + c1) + c2) + c3, which is the order of
// backproject_item (wave w takes views w, w + 4, ...): the sums are the same
// bits under either kernel.  The per-piece arithmetic is backproject_item's.
template <bool EXACT, bool EC, int PMAX, int GW>
__device__ __forceinline__ void backproject_shared_item(const DevGeom &G, const int ngroups, const int nkchunks,
                                                        const int kp, const int winCap, const int item,
                                                        float *smem, const float *__restrict__ proj,
                                                        float *__restrict__ vol)
{
    constexpr int KP = kBackPasses;
    constexpr int CPW = GW / kWaves;                 // columns per wave
    const int kch = item % nkchunks;
    const int t = item / nkchunks;
    const int q = t % ngroups;
    const int j = t / ngroups;
    const int i0 = q * GW;
    const int k0 = kch * kWave * kp;
    const int tid = threadIdx.x, lane = tid & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int kmax = min(k0 + kWave * kp, G.n3) - 1;
    const float a3f = (float)G.a3;
    const bool raw = G.raw_volume != 0;
    const int ncv = min(GW, G.n1 - i0);

    // LDS: records [GW][PMAX][12], piece counts [GW], window bounds per wave
    // [4][4], then the window
    float *rec = smem;
    int *npv = reinterpret_cast<int *>(rec + GW * PMAX * kRecFloats);
    int *bnd = npv + GW;
    float *win = rec + ((GW * PMAX * kRecFloats + GW + 16 + 3) / 4) * 4;

    float acc[4][KP][CPW];
#pragma unroll
    for (int cl = 0; cl < 4; ++cl)
#pragma unroll
        for (int ps = 0; ps < KP; ++ps)
#pragma unroll
            for (int c = 0; c < CPW; ++c) acc[cl][ps][c] = 0.0f;

    for (int view = 0; view < G.nviews; ++view) {
        const int cl = view & 3;
        const ViewGeom V = G.views[(size_t)view * G.vstride];
        const float c2f = (float)V.c2;
        // the view's records of the stack
        {
            const size_t col0 = ((size_t)view * G.vstride * G.n2 + j) * G.n1 + i0;
            const int tp = G.rtab_pmax;
            const float4 *src = reinterpret_cast<const float4 *>(G.rtab + col0 * tp * kRecFloats);
            constexpr int F4 = kRecFloats / 4;
            for (int q4 = tid; q4 < ncv * tp * F4; q4 += kBlock) {
                const int cs = q4 / F4, c = cs / tp, sl = cs - c * tp;
                reinterpret_cast<float4 *>(rec)[(c * PMAX + sl) * F4 + (q4 - cs * F4)] = src[q4];
            }
            if (tid < GW) npv[tid] = tid < ncv ? G.rtab_n[col0 + tid] : 0;
        }
        __syncthreads();
        // the window: columns of all pieces, rows from the chunk's top voxel
        // (smallest chi2) to its bottom voxel
        {
            int wu0 = 1 << 30, wu1 = -1, wv0 = 1 << 30, wv1 = -1;
            const int c = tid % GW, sl = tid / GW;
            if (sl < PMAX && sl < npv[c]) {
                const float *r = rec + (c * PMAX + sl) * kRecFloats;
                const int u = __float_as_int(r[0]);
                const float beta = r[6], mfac = r[10];
                const float Ytop_hi = fmaf(-(float)kmax, r[4], r[2]) + fmaf(-(float)kmax, r[5], r[3]);
                const float Ytop_lo = fmaf(-(float)k0, r[4], r[2]) + fmaf(-(float)k0, r[5], r[3]);
                int a, b, a2, b2;
                row_range<EC>(Ytop_hi, beta, mfac, c2f, G.N, a, b);
                row_range<EC>(Ytop_lo, beta, mfac, c2f, G.N, a2, b2);
                wu0 = u;
                wu1 = u;
                wv0 = min(a, a2);
                wv1 = max(b, b2);
            }
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                wu0 = min(wu0, __shfl_xor(wu0, off));
                wu1 = max(wu1, __shfl_xor(wu1, off));
                wv0 = min(wv0, __shfl_xor(wv0, off));
                wv1 = max(wv1, __shfl_xor(wv1, off));
            }
            if (lane == 0) {
                bnd[wave * 4] = wu0;
                bnd[wave * 4 + 1] = wu1;
                bnd[wave * 4 + 2] = wv0;
                bnd[wave * 4 + 3] = wv1;
            }
        }
        __syncthreads();
        int wu0 = bnd[0], wu1 = bnd[1], wv0 = bnd[2], wv1 = bnd[3];
#pragma unroll
        for (int w = 1; w < kWaves; ++w) {
            wu0 = min(wu0, bnd[w * 4]);
            wu1 = max(wu1, bnd[w * 4 + 1]);
            wv0 = min(wv0, bnd[w * 4 + 2]);
            wv1 = max(wv1, bnd[w * 4 + 3]);
        }
        wu0 = __builtin_amdgcn_readfirstlane(wu0);
        wu1 = __builtin_amdgcn_readfirstlane(wu1);
        wv0 = __builtin_amdgcn_readfirstlane(wv0);
        wv1 = __builtin_amdgcn_readfirstlane(wv1);
        if (wu1 < wu0 || wv1 < wv0) {      // no piece in this view
            __syncthreads();
            continue;
        }
        // one spare row each side absorbs FP32 rounding of intermediate k
        wv0 = max(wv0 - 1, 0);
        wv1 = min(wv1 + 1, G.N - 1);
        const int Wd = wu1 - wu0 + 1;
        const int H = wv1 - wv0 + 1;
        const int Hp = H | 1;
        const float *pv = proj + (size_t)view * G.vstride * G.N * G.M;
        const float *sgv = G.sigma ? G.sigma + (size_t)view * G.vstride * G.sigma_views * G.N * G.M : nullptr;
        const bool useWin = Wd * Hp <= winCap;
        if (useWin) {
            for (int idx = tid; idx < Wd * H; idx += kBlock) {
                const int uu = idx % Wd, vv = idx / Wd;
                const size_t off = (size_t)(wv0 + vv) * G.M + (wu0 + uu);
                float val = pv[off];
                if (sgv) val *= sgv[off];
                win[uu * Hp + vv] = val;
            }
        }
        __syncthreads();

        auto gather = [&](auto winTag) {
            constexpr bool WIN = decltype(winTag)::value;
#pragma unroll
            for (int ps = 0; ps < KP; ++ps) {
                if (ps >= kp || k0 + ps * kWave >= G.n3) break;   // unused pass
                const int k = k0 + ps * kWave + lane;
                const bool kv = k < G.n3;
                const float kf = (float)k;
                const float zt = fmaf(kf, a3f, (float)(G.x3lo + G.a3 - V.s3));
                const float zc = zt - 0.5f * a3f;
#pragma unroll
                for (int cc = 0; cc < CPW; ++cc) {
                    const int c = wave * CPW + cc;
                    const int np = npv[c];
                    if (np == 0) continue;
                    const float *rc = rec + c * PMAX * kRecFloats;
                    float base = 1.0f;
                    if (!EXACT && !raw) base = __builtin_amdgcn_rcpf(fmaf(zc, zc, rc[8]));
                    float a = 0.0f;
                    for (int p = 0; p < np; ++p) {
                        const float4 r0 = *reinterpret_cast<const float4 *>(rc + p * kRecFloats);
                        const float4 r1 = *reinterpret_cast<const float4 *>(rc + p * kRecFloats + 4);
                        const float4 r2 = *reinterpret_cast<const float4 *>(rc + p * kRecFloats + 8);
                        const int u = __float_as_int(r0.x);
                        const float Yh = fmaf(-kf, r1.x, r0.z);
                        const float Yl = fmaf(-kf, r1.y, r0.w);
                        const float Ybl = Yl + r1.y;
                        const float beta = r1.z, rho = r1.w, rho4 = 4.0f * r1.w;
                        int vlo0, vhi0;
                        row_range_unclipped<EC>(Yh + Yl, beta, r2.z, c2f, vlo0, vhi0);
                        const bool ends = !EC || rho < 0.9f;
                        const int vlo = max(max(vlo0, 0), wv0);
                        const int vhi = kv ? min(min(vhi0, G.N - 1), wv1) : vlo - 1;
                        const float *wcol = win + (u - wu0) * Hp - wv0;
                        const float tb = (float)vlo - 0.5f;
                        float d = Yh - tb;
                        float d0 = d + r1.x;         // Ybh - tb, exact on the 2^-10 grid
                        float tc = tb - c2f;
                        float s1p, mp, phip;
                        if (vlo != vlo0 || !ends) boundary<EC>(d, Yl, d0, Ybl, tc, rho, rho4, s1p, mp, phip);
                        else boundary<false>(d, Yl, d0, Ybl, tc, rho, rho4, s1p, mp, phip);
                        float psip = mp + phip;
                        float ap = 0.0f;
                        auto row = [&](float val) {
                            d -= 1.0f;
                            d0 -= 1.0f;
                            tc += 1.0f;
                            float s1n, mn, phin;
                            boundary<EC>(d, Yl, d0, Ybl, tc, rho, rho4, s1n, mn, phin);
                            float w = psip - phin;
                            if (EXACT && !raw) {
                                float mm = 0.5f * (fmaxf(0.0f, -s1p) + fminf(beta, -s1n));
                                mm = fminf(fmaxf(mm, 0.0f), beta);
                                const float zb = fmaf(-mm, r2.y, zt);
                                w *= __builtin_amdgcn_rcpf(fmaf(zb, zb, r2.w));
                            }
                            ap = fmaf(w, val, ap);
                            psip = mn + phin;
                            s1p = s1n;
                        };
                        if (WIN) {
                            const float *const last = wcol + vhi;
                            for (const float *qq = wcol + vlo; qq < last; ++qq) row(*qq);
                            if (vlo <= vhi) {
                                d -= 1.0f;
                                d0 -= 1.0f;
                                tc += 1.0f;
                                float s1n = d + Yl, phin = 0.0f;
                                if (vhi != vhi0 || !ends) {
                                    float mn;
                                    boundary<EC>(d, Yl, d0, Ybl, tc, rho, rho4, s1n, mn, phin);
                                }
                                float w = psip - phin;
                                if (EXACT && !raw) {
                                    float mm = 0.5f * (fmaxf(0.0f, -s1p) + fminf(beta, -s1n));
                                    mm = fminf(fmaxf(mm, 0.0f), beta);
                                    const float zb = fmaf(-mm, r2.y, zt);
                                    w *= __builtin_amdgcn_rcpf(fmaf(zb, zb, r2.w));
                                }
                                ap = fmaf(w, *last, ap);
                            }
                        } else {
                            for (int v = vlo; v <= vhi; ++v) {
                                const size_t off = (size_t)v * G.M + u;
                                float val = pv[off];
                                if (sgv) val *= sgv[off];
                                row(val);
                            }
                        }
                        a = fmaf(base * r0.y, ap, a);
                    }
                    // the partial sum of view class cl (a uniform index)
#pragma unroll
                    for (int ccl = 0; ccl < 4; ++ccl)
                        if (ccl == cl) acc[ccl][ps][cc] += a;
                }
            }
        };
        if (useWin) gather(std::true_type{});
        else gather(std::false_type{});
        __syncthreads();                   // the next view reuses the records and the window
    }

    // ((c0 + c1) + c2) + c3 per voxel, one store each
#pragma unroll
    for (int ps = 0; ps < KP; ++ps) {
        if (ps >= kp) break;
        const int k = k0 + ps * kWave + lane;
#pragma unroll
        for (int cc = 0; cc < CPW; ++cc) {
            const int i = i0 + wave * CPW + cc;
            float sum = acc[0][ps][cc];
#pragma unroll
            for (int w = 1; w < 4; ++w) sum += acc[w][ps][cc];
            if (k < G.n3 && i < G.n1) vol[((size_t)k * G.n2 + j) * G.n1 + i] = sum;
        }
    }
}

template <bool EXACT, bool EC, int PMAX, int GW>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3)))
backproject_shared_kernel(const DevGeom G, const int ngroups, const int nkchunks, const int kp, const int items,
                          const int chunk, const int winCap, const float *__restrict__ proj,
                          float *__restrict__ vol, const double *__restrict__ stop)
{
    extern __shared__ __align__(16) float smem[];
    if (stop && *stop != 0.0) return;
    const int item = (blockIdx.x & 7) * chunk + (blockIdx.x >> 3);
    if (item >= items) return;
    backproject_shared_item<EXACT, EC, PMAX, GW>(G, ngroups, nkchunks, kp, winCap, item, smem, proj, vol);
}

// ------------------------------------------------------------ batched, persistent

// Next work item of a persistent workgroup (one atomic per item) and the
// problem it belongs to; segments are ordered largest items first.
__device__ __forceinline__ bool next_item(const BatchTable &T, int *counter, int &p, int &local)
{
    __shared__ int s_item;
    __syncthreads();   // the previous item's LDS use is over
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
    __syncthreads();
    const int item = __builtin_amdgcn_readfirstlane(s_item);   // uniform: scalar loads below
    if (item >= T.start[T.n]) return false;
    int seg = 0;
    while (T.start[seg + 1] <= item) ++seg;
    p = __builtin_amdgcn_readfirstlane(T.order[seg]);
    local = item - T.start[seg];
    return true;
}

template <bool EXACT, bool EC, bool TAB = false>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(5)))
project_batched_kernel(const BatchProblem *__restrict__ probs, const BatchTable *__restrict__ T,
                       int *counter)
{
    extern __shared__ __align__(16) float smem[];
    int p, local;
    while (next_item(*T, counter, p, local)) {
        const BatchProblem &P = probs[p];
        if (P.stop && *P.stop != 0.0) continue;
        if (P.pmax <= 4)
            project_item<EXACT, EC, 4, false, TAB>(P.G, P.U, local, smem, P.in, P.out, P.gmax);
        else
            project_item<EXACT, EC, 8, false, TAB>(P.G, P.U, local, smem, P.in, P.out, P.gmax);
    }
}

// One persistent launch per (stack width GW, piece stride PMAX) present in a
// batch, over the members with that width and stride; each problem keeps its
// own passes and window.
// Backprojection sums do not depend on the plan, so every problem's result
// equals its own single-problem launch bitwise, and each kernel holds a
// single variant of the gather (its registers fit like the single-problem
// kernel's; one kernel inlining every variant spilled).
template <bool EXACT, bool EC, int PMAX, int GW, bool TAB = false>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3)))
backproject_batched_kernel(const BatchProblem *__restrict__ probs, const BatchTable *__restrict__ T,
                           int *counter)
{
    extern __shared__ __align__(16) float smem[];
    int p, local;
    while (next_item(*T, counter, p, local)) {
        const BatchProblem &P = probs[p];
        if (P.stop && *P.stop != 0.0) continue;
        backproject_item<EXACT, EC, PMAX, GW, false, TAB>(P.G, P.ngroups, P.nkchunks, P.kp, P.win_cap, local, smem,
                                                         P.in, P.out);
    }
}

// Per-call setup of a batched launch (a kernel, so it can sit in a graph):
// the I/O pointers of every problem and a zeroed work counter.
__global__ void batch_setup(BatchProblem *probs, const BatchIO io, int *counter)
{
    if (threadIdx.x != 0) return;
#pragma unroll
    for (int q = 0; q < kMaxBatch; ++q) {
        if (q < io.n) {
            probs[q].in = io.in[q];
            probs[q].out = io.out[q];
            probs[q].G.sigma = io.sigma[q];
            probs[q].G.raw_volume = io.raw;
            probs[q].stop = io.stop[q];
        }
    }
    *counter = 0;
}

template <bool EXACT, bool EC, bool TT = false>
hipError_t launch_p(const DevGeom &g, const ProjLaunch &L, const float *vol, float *proj,
                    unsigned *gmax, hipStream_t s, const double *stop)
{
    if (gmax) {
        hipError_t e = launch_group_max(g, vol, gmax, s, stop);
        if (e != hipSuccess) return e;
    }
    const dim3 grid(8 * L.chunk), block(kBlock);
    if (!TT && g.rtab) {
        // the geometry's cached records
        if (g.rtab_pmax != (L.pmax <= 4 ? 4 : 8)) return hipErrorInvalidValue;
        if (L.pmax <= 4)
            hipLaunchKernelGGL((project_kernel<EXACT, EC, 4, false, true>), grid, block, L.lds, s, g, L.U, L.nbands,
                               vol, proj, gmax, stop);
        else
            hipLaunchKernelGGL((project_kernel<EXACT, EC, 8, false, true>), grid, block, L.lds, s, g, L.U, L.nbands,
                               vol, proj, gmax, stop);
        return hipGetLastError();
    }
    if (L.pmax <= 4)
        hipLaunchKernelGGL((project_kernel<EXACT, EC, 4, TT>), grid, block, L.lds, s, g, L.U, L.nbands, vol, proj,
                           gmax, stop);
    else
        hipLaunchKernelGGL((project_kernel<EXACT, EC, 8, TT>), grid, block, L.lds, s, g, L.U, L.nbands, vol, proj,
                           gmax, stop);
    return hipGetLastError();
}

template <bool EXACT, bool EC, int PMAX, bool TT = false, bool TAB = false>
hipError_t launch_bp_gw(const DevGeom &g, const BackLaunch &L, const float *proj, float *vol,
                        hipStream_t s, const double *stop)
{
    const dim3 grid(8 * L.chunk), block(kBlock);
    switch (L.gw) {
    case 16:
        hipLaunchKernelGGL((backproject_kernel<EXACT, EC, PMAX, 16, TT, TAB>), grid, block, L.lds, s, g,
                           L.ngroups, L.nkchunks, L.kp, L.items, L.chunk, L.win_cap, proj, vol, stop);
        break;
    case 8:
        hipLaunchKernelGGL((backproject_kernel<EXACT, EC, PMAX, 8, TT, TAB>), grid, block, L.lds, s, g,
                           L.ngroups, L.nkchunks, L.kp, L.items, L.chunk, L.win_cap, proj, vol, stop);
        break;
    default:
        hipLaunchKernelGGL((backproject_kernel<EXACT, EC, PMAX, 4, TT, TAB>), grid, block, L.lds, s, g,
                           L.ngroups, L.nkchunks, L.kp, L.items, L.chunk, L.win_cap, proj, vol, stop);
        break;
    }
    return hipGetLastError();
}

template <bool EXACT, bool EC, int PMAX>
hipError_t launch_bp_shared(const DevGeom &g, const BackLaunch &L, const float *proj, float *vol,
                            hipStream_t s, const double *stop)
{
    const dim3 grid(8 * L.chunk), block(kBlock);
    switch (L.gw) {
    case 16:
        hipLaunchKernelGGL((backproject_shared_kernel<EXACT, EC, PMAX, 16>), grid, block, L.lds, s, g, L.ngroups,
                           L.nkchunks, L.kp, L.items, L.chunk, L.win_cap, proj, vol, stop);
        break;
    case 8:
        hipLaunchKernelGGL((backproject_shared_kernel<EXACT, EC, PMAX, 8>), grid, block, L.lds, s, g, L.ngroups,
                           L.nkchunks, L.kp, L.items, L.chunk, L.win_cap, proj, vol, stop);
        break;
    default:
        hipLaunchKernelGGL((backproject_shared_kernel<EXACT, EC, PMAX, 4>), grid, block, L.lds, s, g, L.ngroups,
                           L.nkchunks, L.kp, L.items, L.chunk, L.win_cap, proj, vol, stop);
        break;
    }
    return hipGetLastError();
}

template <bool EXACT, bool EC, bool TT = false>
hipError_t launch_bp(const DevGeom &g, const BackLaunch &L, const float *proj, float *vol,
                     hipStream_t s, const double *stop)
{
    if (!TT && g.rtab) {
        // the geometry's cached records (the plan L was made for these kernels)
        if (L.pmax > 8 || g.rtab_pmax != (L.pmax <= 4 ? 4 : 8)) return hipErrorInvalidValue;
        if (L.shared) {
            if (L.pmax <= 4) return launch_bp_shared<EXACT, EC, 4>(g, L, proj, vol, s, stop);
            return launch_bp_shared<EXACT, EC, 8>(g, L, proj, vol, s, stop);
        }
        if (L.pmax <= 4) return launch_bp_gw<EXACT, EC, 4, false, true>(g, L, proj, vol, s, stop);
        return launch_bp_gw<EXACT, EC, 8, false, true>(g, L, proj, vol, s, stop);
    }
    if (L.pmax <= 4) return launch_bp_gw<EXACT, EC, 4, TT>(g, L, proj, vol, s, stop);
    if (L.pmax <= 8) return launch_bp_gw<EXACT, EC, 8, TT>(g, L, proj, vol, s, stop);
    // wide footprints: 4-column stacks only
    if (L.gw != 4) return hipErrorInvalidValue;
    hipLaunchKernelGGL((backproject_kernel<EXACT, EC, kPmaxWide, 4, TT>), dim3(8 * L.chunk), dim3(kBlock), L.lds, s, g,
                       L.ngroups, L.nkchunks, L.kp, L.items, L.chunk, L.win_cap, proj, vol, stop);
    return hipGetLastError();
}

template <bool EXACT, bool EC, int PMAX, bool TT = false, bool TAB = false>
hipError_t set_lds_one(size_t n)
{
    hipError_t e = hipFuncSetAttribute((const void *)project_kernel<EXACT, EC, PMAX, TT, TAB>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)n);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)backproject_kernel<EXACT, EC, PMAX, 16, TT, TAB>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)n);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)backproject_kernel<EXACT, EC, PMAX, 8, TT, TAB>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)n);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)backproject_kernel<EXACT, EC, PMAX, 4, TT, TAB>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)n);
    if constexpr (TAB && !TT) {
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void *)backproject_shared_kernel<EXACT, EC, PMAX, 16>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)n);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void *)backproject_shared_kernel<EXACT, EC, PMAX, 8>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)n);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void *)backproject_shared_kernel<EXACT, EC, PMAX, 4>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)n);
    }
    return e;
}

template <bool EXACT, bool EC, bool TT = false>
hipError_t set_lds_wide(size_t n)
{
    return hipFuncSetAttribute((const void *)backproject_kernel<EXACT, EC, kPmaxWide, 4, TT>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)n);
}

template <bool EXACT, bool EC, bool TAB>
hipError_t launch_pb(BatchProblem *probs, const BatchTable *tab, int *counter, int grid, size_t lds,
                     hipStream_t s)
{
    hipLaunchKernelGGL((project_batched_kernel<EXACT, EC, TAB>), dim3(grid), dim3(kBlock), lds, s, probs, tab,
                       counter);
    return hipGetLastError();
}

template <bool EXACT, bool EC, int PMAX, bool TAB>
hipError_t launch_bb_p(BatchProblem *probs, const BatchTable *tab, int *counter, int grid, size_t lds, int gw,
                       hipStream_t s)
{
    if (gw == 16)
        hipLaunchKernelGGL((backproject_batched_kernel<EXACT, EC, PMAX, 16, TAB>), dim3(grid), dim3(kBlock), lds, s,
                           probs, tab, counter);
    else if (gw == 8)
        hipLaunchKernelGGL((backproject_batched_kernel<EXACT, EC, PMAX, 8, TAB>), dim3(grid), dim3(kBlock), lds, s,
                           probs, tab, counter);
    else
        hipLaunchKernelGGL((backproject_batched_kernel<EXACT, EC, PMAX, 4, TAB>), dim3(grid), dim3(kBlock), lds, s,
                           probs, tab, counter);
    return hipGetLastError();
}

template <bool EXACT, bool EC, bool TAB>
hipError_t launch_bb(BatchProblem *probs, const BatchTable *tab, int *counter, int grid, size_t lds, int gw, int pmax,
                     hipStream_t s)
{
    return pmax <= 4 ? launch_bb_p<EXACT, EC, 4, TAB>(probs, tab, counter, grid, lds, gw, s)
                     : launch_bb_p<EXACT, EC, 8, TAB>(probs, tab, counter, grid, lds, gw, s);
}

template <bool EXACT, bool EC, int PMAX, bool TAB>
hipError_t set_lds_batched_back(size_t n)
{
    hipError_t e = hipFuncSetAttribute((const void *)backproject_batched_kernel<EXACT, EC, PMAX, 16, TAB>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)n);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)backproject_batched_kernel<EXACT, EC, PMAX, 8, TAB>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)n);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)backproject_batched_kernel<EXACT, EC, PMAX, 4, TAB>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)n);
    return e;
}

template <bool EXACT, bool EC, bool TAB>
hipError_t set_lds_batched(size_t n)
{
    hipError_t e = hipFuncSetAttribute((const void *)project_batched_kernel<EXACT, EC, TAB>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)n);
    if (e == hipSuccess) e = set_lds_batched_back<EXACT, EC, 4, TAB>(n);
    if (e == hipSuccess) e = set_lds_batched_back<EXACT, EC, 8, TAB>(n);
    return e;
}

template <bool TAB>
hipError_t launch_batched_t(bool backward, BatchProblem *probs, const BatchTable *tab, int *counter, bool exact,
                            bool ec, int grid, size_t lds, int gw, int pmax, hipStream_t s)
{
    if (!backward) {
        if (exact) return ec ? launch_pb<true, true, TAB>(probs, tab, counter, grid, lds, s)
                             : launch_pb<true, false, TAB>(probs, tab, counter, grid, lds, s);
        return ec ? launch_pb<false, true, TAB>(probs, tab, counter, grid, lds, s)
                  : launch_pb<false, false, TAB>(probs, tab, counter, grid, lds, s);
    }
    if (exact) return ec ? launch_bb<true, true, TAB>(probs, tab, counter, grid, lds, gw, pmax, s)
                         : launch_bb<true, false, TAB>(probs, tab, counter, grid, lds, gw, pmax, s);
    return ec ? launch_bb<false, true, TAB>(probs, tab, counter, grid, lds, gw, pmax, s)
              : launch_bb<false, false, TAB>(probs, tab, counter, grid, lds, gw, pmax, s);
}

template <int PMAX, bool TAB>
const void *back_batched_fn(int gw)
{
    if (gw == 16) return (const void *)backproject_batched_kernel<false, true, PMAX, 16, TAB>;
    if (gw == 8) return (const void *)backproject_batched_kernel<false, true, PMAX, 8, TAB>;
    return (const void *)backproject_batched_kernel<false, true, PMAX, 4, TAB>;
}

template <bool TAB>
int blocks_per_cu_t(bool backward, size_t lds, int gw, int pmax)
{
    int nb = 0;
    const void *fn = !backward ? (const void *)project_batched_kernel<false, true, TAB>
                               : pmax <= 4 ? back_batched_fn<4, TAB>(gw) : back_batched_fn<8, TAB>(gw);
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, kBlock, lds);
    if (e != hipSuccess || nb < 1) nb = 1;
    return nb;
}

}  // namespace

hipError_t launch_batched(bool backward, BatchProblem *probs, const BatchTable *tab, int *counter,
                          const BatchIO &io, bool exact, bool ec, int grid, size_t lds, int gw, int pmax, bool cached,
                          hipStream_t s)
{
    hipLaunchKernelGGL(batch_setup, dim3(1), dim3(64), 0, s, probs, io, counter);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return cached ? launch_batched_t<true>(backward, probs, tab, counter, exact, ec, grid, lds, gw, pmax, s)
                  : launch_batched_t<false>(backward, probs, tab, counter, exact, ec, grid, lds, gw, pmax, s);
}

// Workgroups of a persistent batched kernel that fit on one CU at this LDS size.
int batched_blocks_per_cu(bool backward, size_t lds, int gw, int pmax, bool cached)
{
    return cached ? blocks_per_cu_t<true>(backward, lds, gw, pmax) : blocks_per_cu_t<false>(backward, lds, gw, pmax);
}

// Allow the dynamic LDS sizes chosen by the host (above the 64 KB default).
hipError_t configure_kernel_lds(size_t max_lds, size_t max_lds_batched)
{
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = set_lds_one<true, true, 4>(max_lds);
    if (e == hipSuccess) e = set_lds_one<true, false, 4>(max_lds);
    if (e == hipSuccess) e = set_lds_one<false, true, 4>(max_lds);
    if (e == hipSuccess) e = set_lds_one<false, false, 4>(max_lds);
    if (e == hipSuccess) e = set_lds_one<true, true, 8>(max_lds);
    if (e == hipSuccess) e = set_lds_one<true, false, 8>(max_lds);
    if (e == hipSuccess) e = set_lds_one<false, true, 8>(max_lds);
    if (e == hipSuccess) e = set_lds_one<false, false, 8>(max_lds);
    if (e == hipSuccess) e = set_lds_wide<true, true>(max_lds);
    if (e == hipSuccess) e = set_lds_wide<true, false>(max_lds);
    if (e == hipSuccess) e = set_lds_wide<false, true>(max_lds);
    if (e == hipSuccess) e = set_lds_wide<false, false>(max_lds);
    if (e == hipSuccess) e = set_lds_one<false, true, 4, true>(max_lds);
    if (e == hipSuccess) e = set_lds_one<false, true, 8, true>(max_lds);
    if (e == hipSuccess) e = set_lds_wide<false, true, true>(max_lds);
    if (e == hipSuccess) e = set_lds_one<true, true, 4, false, true>(max_lds);
    if (e == hipSuccess) e = set_lds_one<true, false, 4, false, true>(max_lds);
    if (e == hipSuccess) e = set_lds_one<false, true, 4, false, true>(max_lds);
    if (e == hipSuccess) e = set_lds_one<false, false, 4, false, true>(max_lds);
    if (e == hipSuccess) e = set_lds_one<true, true, 8, false, true>(max_lds);
    if (e == hipSuccess) e = set_lds_one<true, false, 8, false, true>(max_lds);
    if (e == hipSuccess) e = set_lds_one<false, true, 8, false, true>(max_lds);
    if (e == hipSuccess) e = set_lds_one<false, false, 8, false, true>(max_lds);
    if (e == hipSuccess) e = set_lds_batched<true, true, false>(max_lds_batched);
    if (e == hipSuccess) e = set_lds_batched<true, false, false>(max_lds_batched);
    if (e == hipSuccess) e = set_lds_batched<false, true, false>(max_lds_batched);
    if (e == hipSuccess) e = set_lds_batched<false, false, false>(max_lds_batched);
    if (e == hipSuccess) e = set_lds_batched<true, true, true>(max_lds_batched);
    if (e == hipSuccess) e = set_lds_batched<true, false, true>(max_lds_batched);
    if (e == hipSuccess) e = set_lds_batched<false, true, true>(max_lds_batched);
    if (e == hipSuccess) e = set_lds_batched<false, false, true>(max_lds_batched);
    return e;
}

hipError_t launch_project(const DevGeom &g, const ProjLaunch &L, int model, bool ec,
                          const float *vol, float *proj, unsigned *gmax, hipStream_t stream, const double *stop)
{
    // TT: its ramps need the row margins of the EC instantiations
    if (model == kModelTT) return launch_p<false, true, true>(g, L, vol, proj, gmax, stream, stop);
    const bool exact = model == kModelExact;
    if (exact) return ec ? launch_p<true, true>(g, L, vol, proj, gmax, stream, stop)
                         : launch_p<true, false>(g, L, vol, proj, gmax, stream, stop);
    return ec ? launch_p<false, true>(g, L, vol, proj, gmax, stream, stop)
              : launch_p<false, false>(g, L, vol, proj, gmax, stream, stop);
}

int64_t group_max_cells(const DevGeom &g)
{
    return (int64_t)g.n2 * ((g.n1 + 15) / 16);
}

hipError_t launch_group_max(const DevGeom &g, const float *vol, unsigned *gmax, hipStream_t stream,
                            const double *stop)
{
    const int64_t cells = group_max_cells(g);
    hipLaunchKernelGGL(group_max_kernel, dim3((unsigned)((cells + kWaves - 1) / kWaves)), dim3(kBlock), 0, stream,
                       g, vol, gmax, stop);
    return hipGetLastError();
}

hipError_t launch_record_table(const DevGeom &g, int pmax, float *rec, int *cnt, hipStream_t stream)
{
    const int64_t n = (int64_t)g.n1 * g.n2 * g.nviews;
    const dim3 grid((unsigned)((n + kBlock - 1) / kBlock)), block(kBlock);
    if (pmax == 4)
        hipLaunchKernelGGL(record_table_kernel<4>, grid, block, 0, stream, g, rec, cnt);
    else if (pmax == 8)
        hipLaunchKernelGGL(record_table_kernel<8>, grid, block, 0, stream, g, rec, cnt);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// Fixed device scratch of the allocation-free projection: the per-group
// maxima table of group_max_kernel, at most kStaticScratchWords words.  Every
// GPU the library runs on holds its own copy until the process ends; host
// code never passes the array's name to a kernel (on the host it is only a
// stand-in for the symbol) but the device address that hipGetSymbolAddress
// returns for the current device.
static __device__ __align__(256) unsigned scratch[kStaticScratchWords];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t static_scratch(unsigned **out)
{
    *out = nullptr;
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = static_cast<unsigned *>(p);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

hipError_t launch_backproject(const DevGeom &g, const BackLaunch &L, int model, bool ec,
                              const float *proj, float *vol, hipStream_t stream, const double *stop)
{
    if (model == kModelTT) return launch_bp<false, true, true>(g, L, proj, vol, stream, stop);
    const bool exact = model == kModelExact;
    if (exact) return ec ? launch_bp<true, true>(g, L, proj, vol, stream, stop)
                         : launch_bp<true, false>(g, L, proj, vol, stream, stop);
    return ec ? launch_bp<false, true>(g, L, proj, vol, stream, stop)
              : launch_bp<false, false>(g, L, proj, vol, stream, stop);
}

}  // namespace cvp
