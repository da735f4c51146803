// C ABI of the cutting voxel projector library: argument validation, FP64
// host geometry, device tables and launch configuration.  See include/cvp.h.
#include "cvp.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "cvp_internal.h"

namespace cvp {
hipError_t configure_kernel_lds(size_t max_lds, size_t max_lds_batched);
constexpr size_t kLdsBudget = 30 * 1024;   // default projection plans: five workgroups per CU (160 KB LDS; 5 x 32 KB did not fit)
constexpr size_t kBackLdsBudget = 52 * 1024;   // backprojection windows: three workgroups per CU
constexpr size_t kBackLdsBudgetWide = 80 * 1024;   // records of up to kPmaxWide pieces per column: two per CU
constexpr size_t kBackLdsBudgetCached = 40 * 1024;   // cached records (no FP64 stage, ~105 VGPRs): four per CU
// cached records, three per CU and larger windows: the default for 8-piece
// records (the 16-problem batch's single launches: 450 against 348 ms at four
// per CU); the autotuner may choose either budget for a geometry
constexpr size_t kLdsMax = 156 * 1024;      // any plan: one workgroup per CU at worst
// LDS the persistent batched kernels hold besides their plan's (the work-item
// slot, one 512-byte allocation granule): their plans leave it out of the
// budget, or four 40 KB workgroups would not fit a CU's 160 KB
constexpr size_t kBatchStaticLds = 512;
constexpr size_t kLdsBatchMax = kLdsMax;
bool plan_projection(int N, int n2, int M, int nviews, int pmax, int force_u, ProjLaunch &L);
bool plan_backprojection(const DevGeom &G, int pmax, double zabs, double Dmin, int force_gw,
                         int force_kp, BackLaunch &L, bool cached = false, size_t reserve = 0, int wpc = 0,
                         bool shared_req = false);
}
using cvp::kLdsBudget;

struct cvp_geometry {
    std::vector<double> angles;
    int device = 0;
    cvp::ViewGeom *d_views = nullptr;
    float *d_sigma[2] = {nullptr, nullptr};   // solid angle, cos
    cvp::DevGeom base{};
    cvp::ProjLaunch pl{};
    cvp::BackLaunch bl{};
    int64_t nvox = 0, npix = 0;
    double zabs = 0.0, Dmin = 0.0;   // for launch planning
    int pmax = 4;                    // pieces per column the kernels keep (4, 8 or kPmaxWide)
    double wone_tt = 0.0, wsum_tt = 0.0;   // fixed-point bounds of the TT projector's weights
    cvp::BackLaunch blc{};           // backprojection plan of the cached-record kernels
    int bp_wpc = 0;                  // requested workgroups per CU of that plan (0: default)
    int bp_shared = 0;               // requested one window per workgroup in that plan
    float *d_rtab = nullptr;         // cached piece records (cvp_geometry_cache_records)
    int *d_rtab_n = nullptr;
    int64_t rtab_bytes = 0;
};

namespace {

thread_local std::string g_err;

cvp_status fail(cvp_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

cvp_status ok()
{
    g_err.clear();
    return CVP_OK;
}

cvp_status device_fail(hipError_t e, const char *what)
{
    if (e == hipErrorOutOfMemory) return fail(CVP_E_NOMEM, "%s: %s", what, hipGetErrorString(e));
    return fail(CVP_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }


// Solid angle of the rectangle [x0,x1] x [y0,y1] on a plane at distance f
// (pixel edges relative to the principal point): the standard arctan form.
double rect_solid_angle(double f, double x0, double x1, double y0, double y1)
{
    auto F = [f](double X, double Y) { return std::atan(X * Y / (f * std::sqrt(X * X + Y * Y + f * f))); };
    return F(x1, y1) - F(x0, y1) - F(x1, y0) + F(x0, y0);
}

}  // namespace

namespace cvp {

size_t project_lds_bytes(int U, int N, int n2, int pmax)
{
    const size_t npad = (size_t)(N | 1);
    (void)pmax;   // piece records live in registers
    // 64-bit band image, row tables, prefix-sum scratch, per-wave maxima
    return (size_t)U * npad * 8 + (size_t)(2 * n2 + 1 + kBlock + kWaves) * 4 + 16;
}

size_t backproject_lds_bytes(int gw, int pmax, int winCap)
{
    const size_t rec = (size_t)back_views_per_pass(gw, pmax) * back_rec_floats(gw, pmax);
    const size_t waveFloats = (rec + winCap + 3) / 4 * 4;
    return kWaves * waveFloats * 4;
}

// Projection: bands of U detector columns (a 64-bit band image of U x N and
// the row tables in LDS).  force_u = 0: U as large as the default LDS budget
// (five workgroups per compute unit) allows; otherwise U = force_u if its LDS
// fits one workgroup.
bool plan_projection(int N, int n2, int M, int nviews, int pmax, int force_u, ProjLaunch &L)
{
    // A work item keeps at most pmax pieces per column, and a column's pieces
    // inside a band of U detector columns are at most U; pmax = 8 with U <= 8
    // therefore serves footprints of any width.
    const int umax = pmax > 8 ? 8 : 32;
    if (pmax > 8) pmax = 8;
    const size_t fixed = project_lds_bytes(0, N, n2, pmax);
    const size_t perU = project_lds_bytes(1, N, n2, pmax) - fixed;
    int U = force_u;
    if (U <= 0) {
        // as wide as the default budget allows; a single column may use more
        if (fixed + perU > kLdsMax) return false;
        U = fixed + perU <= kLdsBudget ? (int)((kLdsBudget - fixed) / perU) : 1;
        U = std::max(1, std::min(U, umax));
    } else if (U > umax || project_lds_bytes(U, N, n2, pmax) > kLdsMax) {
        return false;
    }
    L.U = U;
    L.nbands = (M + U - 1) / U;
    L.items = L.nbands * nviews;
    L.chunk = nviews * ((L.nbands + 7) / 8);   // work items per XCD (bands interleaved over XCDs)
    L.pmax = pmax;
    L.lds = project_lds_bytes(U, N, n2, pmax);
    return true;
}

// Backprojection: stacks of GW columns x 64 kp voxels; the largest stack whose
// estimated detector window fits the per-wave LDS window (force_gw > 0 and
// force_kp > 0 fix them).
bool plan_backprojection(const DevGeom &G, int pmax, double zabs, double Dmin, int force_gw,
                         int force_kp, BackLaunch &L, bool cached, size_t reserve, int wpc, bool shared_req)
{
    const double mag = G.f / Dmin;
    // (stack width, passes) by stack area; the first whose estimated window
    // fits the per-wave LDS window, else the last admissible one (its windows
    // are then read from global memory)
    // (wide footprints: records of kPmaxWide pieces, 4-column stacks only)
    static const int cands[6][2] = {{16, 2}, {16, 1}, {8, 2}, {8, 1}, {4, 2}, {4, 1}};
    // the first candidate whose window fits the budget (true), else the last
    // admissible one (false), gw = 0 if none is
    auto choose = [&](size_t budget, int &gw, int &kp, int &cap) {
        gw = kp = cap = 0;
        for (const auto &cd : cands) {
            const int cand = cd[0], ckp = cd[1];
            if ((force_gw > 0 && cand != force_gw) || (force_kp > 0 && ckp != force_kp)) continue;
            if (pmax > 8 && cand != 4) continue;
            const size_t rec = (size_t)back_views_per_pass(cand, pmax) * back_rec_floats(cand, pmax);
            if (rec * kWaves * 4 >= budget) continue;
            const int c = (int)((budget / (kWaves * 4) - rec) / 4 * 4);
            if (!cached && c < kBackPasses * cand * 64) continue;   // the window area also parks the accumulators
            if (c < 1024) continue;
            const double wu = std::hypot(cand * G.a1, G.a2) * mag / G.b1 + pmax + 2;
            const double zspan = std::hypot(cand * G.a1, G.a2);
            const double wv = 64 * ckp * G.a3 * mag / G.b2 + zabs * (G.f / G.b2) * zspan / (Dmin * Dmin) + 6;
            gw = cand;
            kp = ckp;
            cap = c;
            if (wu * ((int)wv | 1) <= c) return true;
        }
        return false;
    };
    // with cached records the kernel needs no FP64 stage and parks nothing:
    // a smaller budget lets four workgroups share a compute unit (the
    // default for 4-piece records) or a larger one keeps larger windows in
    // LDS with three (8-piece records)
    if (pmax > 8) wpc = 2;
    else if (!cached) wpc = 3;
    else if (wpc != 3 && wpc != 4) wpc = pmax > 4 ? 3 : 4;
    const size_t budget = (pmax > 8 ? kBackLdsBudgetWide
                           : cached && wpc == 4 ? kBackLdsBudgetCached : kBackLdsBudget) - reserve;
    int gw = 0, kp = 0, cap = 0, shared = 0;
    if (shared_req && cached && pmax <= 8) {
        // one window per workgroup (all four waves on one view), for stacks of
        // 8 or 16 columns: the first whose window fits it, else the last one
        for (const auto &cd : cands) {
            const int cand = cd[0], ckp = cd[1];
            if ((force_gw > 0 && cand != force_gw) || (force_kp > 0 && ckp != force_kp) || cand < 8) continue;
            const size_t rec = (size_t)((cand * pmax * kRecFloats + cand + 16 + 3) / 4 * 4) * 4;
            if (rec + 4096 >= budget) continue;
            const int c = (int)((budget - rec) / 4 / 4 * 4);
            const double wu = std::hypot(cand * G.a1, G.a2) * mag / G.b1 + pmax + 2;
            const double zspan = std::hypot(cand * G.a1, G.a2);
            const double wv = 64 * ckp * G.a3 * mag / G.b2 + zabs * (G.f / G.b2) * zspan / (Dmin * Dmin) + 6;
            gw = cand;
            kp = ckp;
            cap = c;
            shared = 1;
            if (wu * ((int)wv | 1) <= c) break;
        }
    }
    if (!shared) choose(budget, gw, kp, cap);
    if (gw == 0) return false;
    L.gw = gw;
    L.kp = kp;
    L.win_cap = cap;
    L.pmax = pmax;
    L.ngroups = (G.n1 + gw - 1) / gw;
    L.nkchunks = (G.n3 + 64 * kp - 1) / (64 * kp);
    L.items = G.n2 * L.ngroups * L.nkchunks;
    L.chunk = (L.items + 7) / 8;
    L.lds = shared ? (size_t)((gw * pmax * kRecFloats + gw + 16 + 3) / 4 * 4) * 4 + (size_t)cap * 4
                   : backproject_lds_bytes(gw, pmax, cap);
    L.wpc = wpc;
    L.shared = shared;
    return true;
}

}  // namespace cvp

extern "C" {

const char *cvp_status_string(cvp_status s)
{
    switch (s) {
    case CVP_OK: return "CVP_OK";
    case CVP_E_INVALID: return "CVP_E_INVALID";
    case CVP_E_NOMEM: return "CVP_E_NOMEM";
    case CVP_E_DEVICE: return "CVP_E_DEVICE";
    case CVP_E_UNSUPPORTED: return "CVP_E_UNSUPPORTED";
    case CVP_E_BREAKDOWN: return "CVP_E_BREAKDOWN";
    }
    return "CVP_E_UNKNOWN";
}

cvp_status cvp_last_error_detail(char *buf, size_t n)
{
    if (!buf) return CVP_E_INVALID;
    if (n == 0) return CVP_OK;
    std::strncpy(buf, g_err.c_str(), n - 1);
    buf[n - 1] = '\0';
    return CVP_OK;
}

void cvp_geometry_destroy(cvp_geometry *g)
{
    if (!g) return;
    if (g->d_views) (void)hipFree(g->d_views);
    for (float *p : g->d_sigma)
        if (p) (void)hipFree(p);
    if (g->d_rtab) (void)hipFree(g->d_rtab);
    if (g->d_rtab_n) (void)hipFree(g->d_rtab_n);
    delete g;
}

}  // extern "C"

namespace {

// Volume and detector of a geometry under construction.
struct VolDet {
    int n1, n2, n3, M, N;
    double a1, a2, a3;
    double x1lo, x2lo, x3lo;
};

cvp_status check_vol_det(const int32_t dims[3], const double vox[3], const double off[3], int cols, int rows,
                         VolDet &vd)
{
    for (int a = 0; a < 3; ++a) {
        if (dims[a] <= 0 || dims[a] > 16384)
            return fail(CVP_E_INVALID, "vol_dims[%d] = %d (must be 1..16384)", a, dims[a]);
        if (!finite_pos(vox[a])) return fail(CVP_E_INVALID, "voxel_mm[%d] must be finite and > 0", a);
        if (!std::isfinite(off[a])) return fail(CVP_E_INVALID, "vol_offset_mm[%d] must be finite", a);
    }
    if (cols <= 0 || cols > 16384) return fail(CVP_E_INVALID, "det_cols = %d (must be 1..16384)", cols);
    if (rows <= 0 || rows > 16384) return fail(CVP_E_INVALID, "det_rows = %d (must be 1..16384)", rows);
    vd.n1 = dims[0]; vd.n2 = dims[1]; vd.n3 = dims[2];
    vd.a1 = vox[0]; vd.a2 = vox[1]; vd.a3 = vox[2];
    vd.x1lo = off[0] - 0.5 * vd.n1 * vd.a1;
    vd.x2lo = off[1] - 0.5 * vd.n2 * vd.a2;
    vd.x3lo = off[2] - 0.5 * vd.n3 * vd.a3;
    vd.M = cols; vd.N = rows;
    return CVP_OK;
}

// Per-pixel factors of the second phase for one view's intrinsics: 1/solid
// angle (eq. cvpus) and f^2 / (a cos^3 theta) (eq. cvp), FP64, stored FP32.
// Pixel edges are taken in units of f ((t - c) / (f/b)).
void pixel_factors(const cvp::ViewGeom &V, int M, int N, float *sa, float *cs)
{
    for (int v = 0; v < N; ++v) {
        const double y0 = (v - 0.5 - V.c2) / V.fb2, y1 = (v + 0.5 - V.c2) / V.fb2, yc = (v - V.c2) / V.fb2;
        for (int u = 0; u < M; ++u) {
            const double x0 = (u - 0.5 - V.c1) / V.fb1, x1 = (u + 0.5 - V.c1) / V.fb1, xc = (u - V.c1) / V.fb1;
            sa[(size_t)v * M + u] = (float)(1.0 / rect_solid_angle(1.0, x0, x1, y0, y1));
            const double R = std::sqrt(xc * xc + yc * yc + 1.0);
            cs[(size_t)v * M + u] = (float)(V.fb1 * V.fb2 * R * R * R);
        }
    }
}

// Planning constants of a circular orbit (closed forms over every angle).
struct Circular {
    double D, f, b1, b2, c1, c2, rmax;
};

// Builds the device tables and launch plans from per-view frames.  circ:
// the orbit's constants (then the pixel factor tables keep the orbit's own
// formulas in mm), or nullptr for general views.
cvp_status finish_geometry(const VolDet &vd, std::vector<cvp::ViewGeom> &views, const Circular *circ,
                           const double *angles, cvp_geometry **out)
{
    const int n1 = vd.n1, n2 = vd.n2, n3 = vd.n3, M = vd.M, N = vd.N;
    const double a1 = vd.a1, a2 = vd.a2, a3 = vd.a3, hd = std::hypot(a1, a2);
    const int V = (int)views.size();
    // nearest depth of the volume in front of each source, farthest distance,
    // height range about each source, widest projected voxel base and the
    // rows the volume reaches
    double Dmin = 1e300, rfar = 0.0, zabs = 0.0, wmax = 0.0, ymax = 0.0, om = 0.0, fb1max = 0.0, fb2max = 0.0;
    for (int v = 0; v < V; ++v) {
        const cvp::ViewGeom &W = views[v];
        double dmin_v = 1e300, z_v = 0.0;
        for (int c = 0; c < 8; ++c) {
            const double x = vd.x1lo + ((c & 1) ? n1 * a1 : 0.0), y = vd.x2lo + ((c & 2) ? n2 * a2 : 0.0);
            const double z = vd.x3lo + ((c & 4) ? n3 * a3 : 0.0);
            const double dep = W.dx * (x - W.s1) + W.dy * (y - W.s2);
            dmin_v = std::min(dmin_v, dep);
            z_v = std::max(z_v, std::fabs(z - W.s3));
            rfar = std::max(rfar, std::sqrt((x - W.s1) * (x - W.s1) + (y - W.s2) * (y - W.s2) + (z - W.s3) * (z - W.s3)));
        }
        if (circ) dmin_v = circ->D - circ->rmax;   // every angle of the orbit
        if (!(dmin_v > hd))
            return fail(CVP_E_INVALID, "view %d: the volume must lie in front of the source by more than a voxel "
                                       "diagonal (nearest depth %g mm)", v, dmin_v);
        Dmin = std::min(Dmin, dmin_v);
        zabs = std::max(zabs, z_v);
        wmax = std::max(wmax, hd * W.fb1 / (dmin_v - 0.5 * hd));
        ymax = std::max(ymax, std::fabs(W.c2) + z_v * W.fb2 / dmin_v + 8.0);
        om = std::max(om, 1.0 / (W.fb1 * W.fb2));
        fb1max = std::max(fb1max, W.fb1);
        fb2max = std::max(fb2max, W.fb2);
    }
    if (circ) {
        zabs = std::max(std::fabs(vd.x3lo), std::fabs(vd.x3lo + n3 * a3));
        rfar = std::hypot(circ->D + circ->rmax, zabs);
        const double Dm = circ->D - circ->rmax;
        wmax = hd * circ->f / (circ->b1 * (Dm - 0.5 * hd));
        ymax = std::fabs(circ->c2) + zabs * circ->f / (circ->b2 * Dm) + 8.0;
        om = circ->b1 * circ->b2 / (circ->f * circ->f);
    }
    const int pieces = (int)std::floor(wmax) + 2;
    if (pieces > cvp::kPmaxWide)
        return fail(CVP_E_UNSUPPORTED, "a voxel base projects onto up to %d detector columns (max %d)", pieces,
                    cvp::kPmaxWide);
    if (ymax > 8000.0)
        return fail(CVP_E_UNSUPPORTED, "the volume projects up to %.0f rows from the detector origin (max 8000)", ymax);

    cvp_geometry *g = new (std::nothrow) cvp_geometry();
    if (!g) return fail(CVP_E_NOMEM, "host allocation");
    if (angles) g->angles.assign(angles, angles + V);
    g->nvox = (int64_t)n1 * n2 * n3;
    g->npix = (int64_t)V * N * M;

    // pixel factor tables: one for views that share their intrinsics, else one per view
    bool shared = true;
    for (int v = 1; v < V && shared; ++v)
        shared = views[v].c1 == views[0].c1 && views[v].c2 == views[0].c2 && views[v].fb1 == views[0].fb1 &&
                 views[v].fb2 == views[0].fb2;
    const int ntab = shared ? 1 : V;
    std::vector<float> sig_sa((size_t)ntab * M * N), sig_cos((size_t)ntab * M * N);
    if (circ) {
        const double c1 = circ->c1, c2 = circ->c2, b1 = circ->b1, b2 = circ->b2, f = circ->f;
        for (int v = 0; v < N; ++v) {
            const double y0 = (v - 0.5 - c2) * b2, y1 = (v + 0.5 - c2) * b2, yc = (v - c2) * b2;
            for (int u = 0; u < M; ++u) {
                const double x0 = (u - 0.5 - c1) * b1, x1 = (u + 0.5 - c1) * b1, xc = (u - c1) * b1;
                sig_sa[(size_t)v * M + u] = (float)(1.0 / rect_solid_angle(f, x0, x1, y0, y1));
                const double R = std::sqrt(xc * xc + yc * yc + f * f);
                sig_cos[(size_t)v * M + u] = (float)(R * R * R / (b1 * b2 * f));
            }
        }
    } else {
        for (int t = 0; t < ntab; ++t)
            pixel_factors(views[t], M, N, sig_sa.data() + (size_t)t * M * N, sig_cos.data() + (size_t)t * M * N);
    }

    hipError_t e = hipGetDevice(&g->device);
    if (e != hipSuccess) { cvp_geometry_destroy(g); return device_fail(e, "hipGetDevice"); }
    e = hipMalloc((void **)&g->d_views, views.size() * sizeof(cvp::ViewGeom));
    if (e == hipSuccess) e = hipMalloc((void **)&g->d_sigma[0], sig_sa.size() * sizeof(float));
    if (e == hipSuccess) e = hipMalloc((void **)&g->d_sigma[1], sig_cos.size() * sizeof(float));
    if (e == hipSuccess) e = hipMemcpy(g->d_views, views.data(), views.size() * sizeof(cvp::ViewGeom), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(g->d_sigma[0], sig_sa.data(), sig_sa.size() * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(g->d_sigma[1], sig_cos.data(), sig_cos.size() * sizeof(float), hipMemcpyHostToDevice);
    if (e != hipSuccess) { cvp_geometry_destroy(g); return device_fail(e, "device tables"); }
    static std::once_flag lds_once;
    static hipError_t lds_err = hipSuccess;
    std::call_once(lds_once, [] { lds_err = cvp::configure_kernel_lds(cvp::kLdsMax, cvp::kLdsBatchMax); });
    if (lds_err != hipSuccess) { cvp_geometry_destroy(g); return device_fail(lds_err, "kernel LDS attribute"); }

    cvp::DevGeom &G = g->base;
    G.n1 = n1; G.n2 = n2; G.n3 = n3; G.M = M; G.N = N; G.nviews = V;
    G.a1 = a1; G.a2 = a2; G.a3 = a3;
    G.x1lo = vd.x1lo; G.x2lo = vd.x2lo; G.x3lo = vd.x3lo;
    // planning values (the kernels read every view's own intrinsics)
    G.fb1 = circ ? circ->f / circ->b1 : fb1max;
    G.fb2 = circ ? circ->f / circ->b2 : fb2max;
    G.b2f = 1.0 / G.fb2;
    G.c1 = views[0].c1; G.c2 = views[0].c2;
    G.f = circ ? circ->f : 1.0;
    G.b1 = G.f / G.fb1; G.b2 = G.f / G.fb2;
    G.views = g->d_views;
    G.vstride = 1;
    G.sigma = nullptr;
    G.sigma_views = shared ? 0 : 1;
    G.raw_volume = 0;
    {
        // Any pixel's summed weight per unit |mu| is at most its solid angle
        // (<= b1 b2 / f^2) times the integral of r^-2 r^2 dr (or of r^2 dr for
        // raw volumes) over the source distances the volume spans; 64 covers
        // the approximations of the cut volumes with a wide margin.
        const double r0 = Dmin, r1 = rfar;
        G.wsum_bound = 64.0 * om * (r1 - r0);
        G.wsum_bound_raw = 64.0 * om * (r1 * r1 * r1 - r0 * r0 * r0) / 3.0;
        // One (voxel, pixel) weight is at most the voxel's cut volume (<= a1
        // a2 a3) over r^2 >= Dmin^2; a factor 2 covers FP32 rounding.
        G.wone_bound = 2.0 * a1 * a2 * a3 / (Dmin * Dmin);
        G.wone_bound_raw = 2.0 * a1 * a2 * a3;
        // TT: a weight is at most the central chord estimate, min(a1/|r1|,
        // a2/|r2|) |r| <= sqrt(2) max(a1, a2) |r| / |r_xy|, and |r| / |r_xy|
        // <= sec = sqrt(1 + (zabs / Dmin)^2); a pixel's sum is at most the
        // rays' path through the volume, rfar - Dmin, times sec (the
        // footprints integrate to the chord, 64 as above).
        const double sec = std::sqrt(1.0 + (zabs / Dmin) * (zabs / Dmin));
        g->wone_tt = 2.0 * std::sqrt(2.0) * std::max(a1, a2) * sec;
        g->wsum_tt = 64.0 * (rfar - Dmin + std::hypot(std::hypot(a1, a2), a3)) * sec;
    }

    // pieces per column the kernels keep: 4, 8, or (4-column backprojection
    // stacks, projection bands of at most 8 columns) kPmaxWide
    const int pmax = pieces <= 4 ? 4 : pieces <= 8 ? 8 : cvp::kPmaxWide;
    g->zabs = zabs;
    g->Dmin = Dmin;
    g->pmax = pmax;
    if (!cvp::plan_projection(N, n2, M, V, pmax, 0, g->pl)) {
        cvp_geometry_destroy(g);
        return fail(CVP_E_UNSUPPORTED, "detector rows (%d) or volume rows (%d) too large for the projection LDS layout", N, n2);
    }
    if (!cvp::plan_backprojection(G, pmax, zabs, Dmin, 0, 0, g->bl)) {
        cvp_geometry_destroy(g);
        return fail(CVP_E_UNSUPPORTED, "backprojection LDS window too small");
    }
    *out = g;
    return ok();
}

// One view from a camera matrix P (row-major 3x4, world mm -> homogeneous
// pixel-index coordinates).  With the sign of P fixed so that the volume
// centre has positive depth and M = P[:, :3] normalised so that its third
// row d has unit length: d must be horizontal; c1 = M1.d, c2 = M2.d;
// M1 - c1 d = (f/b1) e1 with e1 horizontal (no skew); M2 - c2 d = -(f/b2) x3
// (chi2 opposite to x3, Sec. III-A); the source is -M^-1 p4.
cvp_status view_from_matrix(const double *Pm, const double ctr[3], int v, cvp::ViewGeom &W)
{
    double P[3][4];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 4; ++c) P[r][c] = Pm[4 * r + c];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 4; ++c)
            if (!std::isfinite(P[r][c])) return fail(CVP_E_INVALID, "matrices[%d] has a non-finite entry", v);
    const double w = P[2][0] * ctr[0] + P[2][1] * ctr[1] + P[2][2] * ctr[2] + P[2][3];
    const double sgn = w < 0.0 ? -1.0 : 1.0;
    const double n3 = std::sqrt(P[2][0] * P[2][0] + P[2][1] * P[2][1] + P[2][2] * P[2][2]);
    if (!(n3 > 0.0) || w == 0.0) return fail(CVP_E_INVALID, "matrices[%d]: degenerate (the volume centre has no depth)", v);
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 4; ++c) P[r][c] *= sgn / n3;
    const double tol = 1e-9;
    const double *d = P[2];
    if (std::fabs(d[2]) > tol)
        return fail(CVP_E_UNSUPPORTED, "matrices[%d]: the principal ray is not horizontal (chi1 would depend on x3, "
                                       "Sec. III-A convention)", v);
    const double c1 = P[0][0] * d[0] + P[0][1] * d[1] + P[0][2] * d[2];
    const double c2 = P[1][0] * d[0] + P[1][1] * d[1] + P[1][2] * d[2];
    const double r1[3] = {P[0][0] - c1 * d[0], P[0][1] - c1 * d[1], P[0][2] - c1 * d[2]};
    const double r2[3] = {P[1][0] - c2 * d[0], P[1][1] - c2 * d[1], P[1][2] - c2 * d[2]};
    const double fb1 = std::hypot(r1[0], r1[1]), fb2 = -r2[2];
    if (!(fb1 > 0.0) || std::fabs(r1[2]) > tol * fb1)
        return fail(CVP_E_UNSUPPORTED, "matrices[%d]: chi1 depends on x3 (skew or tilted columns; Sec. III-A "
                                       "convention)", v);
    if (!(fb2 > 0.0))
        return fail(CVP_E_UNSUPPORTED, "matrices[%d]: chi2 must run opposite to x3 (Sec. III-A convention)", v);
    if (std::hypot(r2[0], r2[1]) > tol * fb2)
        return fail(CVP_E_UNSUPPORTED, "matrices[%d]: chi2 depends on the horizontal position at fixed depth "
                                       "(rolled detector)", v);
    // source: M s = -p4 (Cramer's rule)
    const double m00 = P[0][0], m01 = P[0][1], m02 = P[0][2], m10 = P[1][0], m11 = P[1][1], m12 = P[1][2];
    const double m20 = P[2][0], m21 = P[2][1], m22 = P[2][2];
    const double det = m00 * (m11 * m22 - m12 * m21) - m01 * (m10 * m22 - m12 * m20) + m02 * (m10 * m21 - m11 * m20);
    if (!(std::fabs(det) > 0.0)) return fail(CVP_E_INVALID, "matrices[%d]: singular 3x3 part", v);
    const double b0 = -P[0][3], b1 = -P[1][3], b2 = -P[2][3];
    W.s1 = (b0 * (m11 * m22 - m12 * m21) - m01 * (b1 * m22 - m12 * b2) + m02 * (b1 * m21 - m11 * b2)) / det;
    W.s2 = (m00 * (b1 * m22 - m12 * b2) - b0 * (m10 * m22 - m12 * m20) + m02 * (m10 * b2 - b1 * m20)) / det;
    W.s3 = (m00 * (m11 * b2 - b1 * m21) - m01 * (m10 * b2 - b1 * m20) + b0 * (m10 * m21 - m11 * m20)) / det;
    W.e1x = r1[0] / fb1; W.e1y = r1[1] / fb1;
    W.dx = d[0]; W.dy = d[1];
    W.c1 = c1; W.c2 = c2;
    W.fb1 = fb1; W.fb2 = fb2; W.ifb2 = 1.0 / fb2;
    return CVP_OK;
}

}  // namespace

extern "C" {

cvp_status cvp_geometry_from_views(const cvp_geometry_desc *d, cvp_geometry **out)
{
    if (!out) return fail(CVP_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!d) return fail(CVP_E_INVALID, "desc is NULL");
    VolDet vd;
    cvp_status st = check_vol_det(d->vol_dims, d->voxel_mm, d->vol_offset_mm, d->det_cols, d->det_rows, vd);
    if (st != CVP_OK) return st;
    if (!finite_pos(d->pitch_mm[0]) || !finite_pos(d->pitch_mm[1]))
        return fail(CVP_E_INVALID, "pitch_mm must be finite and > 0");
    if (!finite_pos(d->source_iso_mm)) return fail(CVP_E_INVALID, "source_iso_mm must be finite and > 0");
    if (!std::isfinite(d->source_det_mm) || !(d->source_det_mm > d->source_iso_mm))
        return fail(CVP_E_INVALID, "source_det_mm must exceed source_iso_mm");
    if (d->n_views < 1) return fail(CVP_E_INVALID, "n_views = %d (must be >= 1)", d->n_views);
    if (!d->angles_rad) return fail(CVP_E_INVALID, "angles_rad is NULL");
    for (int v = 0; v < d->n_views; ++v)
        if (!std::isfinite(d->angles_rad[v])) return fail(CVP_E_INVALID, "angles_rad[%d] is not finite", v);
    double c1 = d->principal_px[0], c2 = d->principal_px[1];
    if (std::isnan(c1)) c1 = 0.5 * (d->det_cols - 1);
    if (std::isnan(c2)) c2 = 0.5 * (d->det_rows - 1);
    if (!std::isfinite(c1) || !std::isfinite(c2)) return fail(CVP_E_INVALID, "principal_px must be finite or NAN");

    // farthest point of the volume box from the rotation axis (x1x2 plane)
    double rmax = 0.0;
    for (int c = 0; c < 4; ++c) {
        const double x = (c & 1) ? vd.x1lo + vd.n1 * vd.a1 : vd.x1lo, y = (c & 2) ? vd.x2lo + vd.n2 * vd.a2 : vd.x2lo;
        rmax = std::max(rmax, std::hypot(x, y));
    }
    const double D = d->source_iso_mm, f = d->source_det_mm;
    if (!(D > rmax * (1.0 + 1e-9)))
        return fail(CVP_E_INVALID, "source_iso_mm = %g must exceed the volume's distance from the axis (%g): the source would enter the volume", D, rmax);
    const double b1 = d->pitch_mm[0], b2 = d->pitch_mm[1];
    if (!(D - rmax > std::hypot(vd.a1, vd.a2)))
        return fail(CVP_E_UNSUPPORTED, "the source passes within a voxel diagonal of the volume");

    // per-view frames (Sec. II-C), FP64
    std::vector<cvp::ViewGeom> views(d->n_views);
    for (int v = 0; v < d->n_views; ++v) {
        const double l = d->angles_rad[v], cl = std::cos(l), sl = std::sin(l);
        cvp::ViewGeom &V = views[v];
        V.s1 = D * cl; V.s2 = D * sl; V.s3 = 0.0;
        V.e1x = -sl; V.e1y = cl;
        V.dx = -cl; V.dy = -sl;
        V.c1 = c1; V.c2 = c2;
        V.fb1 = f / b1; V.fb2 = f / b2; V.ifb2 = b2 / f;
    }
    const Circular circ{D, f, b1, b2, c1, c2, rmax};
    return finish_geometry(vd, views, &circ, d->angles_rad, out);
}

cvp_status cvp_geometry_from_matrices(const cvp_geometry_matrices_desc *d, cvp_geometry **out)
{
    if (!out) return fail(CVP_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!d) return fail(CVP_E_INVALID, "desc is NULL");
    VolDet vd;
    cvp_status st = check_vol_det(d->vol_dims, d->voxel_mm, d->vol_offset_mm, d->det_cols, d->det_rows, vd);
    if (st != CVP_OK) return st;
    if (d->n_views < 1) return fail(CVP_E_INVALID, "n_views = %d (must be >= 1)", d->n_views);
    if (!d->matrices) return fail(CVP_E_INVALID, "matrices is NULL");
    std::vector<cvp::ViewGeom> views(d->n_views);
    for (int v = 0; v < d->n_views; ++v) {
        st = view_from_matrix(d->matrices + (size_t)12 * v, d->vol_offset_mm, v, views[v]);
        if (st != CVP_OK) return st;
    }
    return finish_geometry(vd, views, nullptr, nullptr, out);
}

cvp_status cvp_geometry_get_launch(const cvp_geometry *g, cvp_launch *out)
{
    if (!g) return fail(CVP_E_INVALID, "geometry is NULL");
    if (!out) return fail(CVP_E_INVALID, "out is NULL");
    out->proj_band_cols = g->pl.U;
    const cvp::BackLaunch &bl = g->d_rtab ? g->blc : g->bl;
    out->bp_stack_cols = bl.gw;
    out->bp_passes = bl.kp;
    out->bp_workgroups_per_cu = bl.wpc;
    out->bp_shared_window = bl.shared;
    return ok();
}

cvp_status cvp_geometry_set_launch(cvp_geometry *g, const cvp_launch *in)
{
    if (!g) return fail(CVP_E_INVALID, "geometry is NULL");
    if (!in) return fail(CVP_E_INVALID, "launch is NULL");
    const int u = in->proj_band_cols, gw = in->bp_stack_cols, kp = in->bp_passes;
    if (u < 0 || u > 32) return fail(CVP_E_INVALID, "launch.proj_band_cols = %d (0 or 1..32)", u);
    if (gw != 0 && gw != 4 && gw != 8 && gw != 16)
        return fail(CVP_E_INVALID, "launch.bp_stack_cols = %d (0, 4, 8 or 16)", gw);
    if (kp < 0 || kp > cvp::kBackPasses) return fail(CVP_E_INVALID, "launch.bp_passes = %d (0, 1 or 2)", kp);
    const int wpc = in->bp_workgroups_per_cu;
    if (wpc != 0 && wpc != 3 && wpc != 4)
        return fail(CVP_E_INVALID, "launch.bp_workgroups_per_cu = %d (0, 3 or 4)", wpc);
    const int shw = in->bp_shared_window;
    if (shw != 0 && shw != 1) return fail(CVP_E_INVALID, "launch.bp_shared_window = %d (0 or 1)", shw);
    const cvp::DevGeom &G = g->base;
    cvp::ProjLaunch pl{};
    cvp::BackLaunch bl{};
    if (!cvp::plan_projection(G.N, G.n2, G.M, G.nviews, g->pmax, u, pl)) {
        if (g->pmax > 8 && u > 8)
            return fail(CVP_E_UNSUPPORTED, "launch.proj_band_cols = %d: voxels span more than 8 detector columns, "
                                           "bands are limited to 8", u);
        return fail(CVP_E_UNSUPPORTED, "launch.proj_band_cols = %d: band image of %zu bytes exceeds the LDS limit", u,
                    cvp::project_lds_bytes(u, G.N, G.n2, g->pl.pmax));
    }
    // the plan of the cutting voxel launches (cached records or not); the
    // in-kernel plan also serves the TT projector, so it is kept valid too
    cvp::BackLaunch blc = g->blc;
    if (g->d_rtab) {
        if (!cvp::plan_backprojection(G, g->pmax, g->zabs, g->Dmin, gw, kp, blc, true, 0, wpc, shw != 0))
            return fail(CVP_E_UNSUPPORTED, "launch.bp_stack_cols = %d, bp_passes = %d, bp_workgroups_per_cu = %d: "
                                           "does not fit LDS", gw, kp, wpc);
        if (!cvp::plan_backprojection(G, g->pmax, g->zabs, g->Dmin, gw, kp, bl) &&
            !cvp::plan_backprojection(G, g->pmax, g->zabs, g->Dmin, 0, 0, bl))
            return fail(CVP_E_UNSUPPORTED, "backprojection plan");
    } else if (!cvp::plan_backprojection(G, g->pmax, g->zabs, g->Dmin, gw, kp, bl)) {
        return fail(CVP_E_UNSUPPORTED, "launch.bp_stack_cols = %d, bp_passes = %d: does not fit LDS", gw, kp);
    }
    g->pl = pl;
    g->bl = bl;
    g->blc = blc;
    g->bp_wpc = wpc;
    g->bp_shared = shw;
    return ok();
}

cvp_status cvp_geometry_sizes(const cvp_geometry *g, int64_t *n_voxels, int64_t *n_pixels_total)
{
    if (!g) return fail(CVP_E_INVALID, "geometry is NULL");
    if (n_voxels) *n_voxels = g->nvox;
    if (n_pixels_total) *n_pixels_total = g->npix;
    return ok();
}

// The kernels' projector model of validated options.
static int model_of(const cvp_options *o)
{
    return o->variant == CVP_TT ? cvp::kModelTT : o->variant == CVP_EXACT ? cvp::kModelExact : cvp::kModelRelaxed;
}

// The backprojection plan of the cached-record kernels: the in-kernel plan's
// stack shape when it fits their smaller LDS budget, else their default.
static void replan_backprojection(cvp_geometry *g)
{
    cvp::BackLaunch bl{};
    if (cvp::plan_backprojection(g->base, g->pmax, g->zabs, g->Dmin, g->bl.gw, g->bl.kp, bl, true, 0, g->bp_wpc,
                                 g->bp_shared != 0) ||
        cvp::plan_backprojection(g->base, g->pmax, g->zabs, g->Dmin, 0, 0, bl, true, 0, g->bp_wpc, g->bp_shared != 0))
        g->blc = bl;
    else
        g->blc = g->bl;
}

// The backprojection plan of a prepared launch: cached records or not.
static const cvp::BackLaunch &back_plan(const cvp_geometry *g, const cvp::DevGeom &G)
{
    return G.rtab ? g->blc : g->bl;
}

cvp_status cvp_geometry_cache_records(cvp_geometry *g, int32_t enable, int64_t *bytes, void *stream)
{
    if (!g) return fail(CVP_E_INVALID, "geometry is NULL");
    if (enable != 0 && enable != 1) return fail(CVP_E_INVALID, "enable = %d (0 or 1)", enable);
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return device_fail(e, "hipGetDevice");
    if (dev != g->device)
        return fail(CVP_E_INVALID, "geometry lives on device %d but device %d is current", g->device, dev);
    if (!enable) {
        if (g->d_rtab) (void)hipFree(g->d_rtab);
        if (g->d_rtab_n) (void)hipFree(g->d_rtab_n);
        g->d_rtab = nullptr;
        g->d_rtab_n = nullptr;
        g->rtab_bytes = 0;
        replan_backprojection(g);
        if (bytes) *bytes = 0;
        return ok();
    }
    if (g->pmax > 8)
        return fail(CVP_E_UNSUPPORTED, "voxels project onto more than 8 detector columns: records are not cached");
    if (!g->d_rtab) {
        const int64_t cols = (int64_t)g->base.nviews * g->base.n2 * g->base.n1;
        const size_t rb = (size_t)cols * g->pmax * cvp::kRecFloats * sizeof(float);
        const size_t nb = (size_t)cols * sizeof(int);
        e = hipMalloc((void **)&g->d_rtab, rb);
        if (e == hipSuccess) e = hipMalloc((void **)&g->d_rtab_n, nb);
        if (e == hipSuccess) e = cvp::launch_record_table(g->base, g->pmax, g->d_rtab, g->d_rtab_n, (hipStream_t)stream);
        if (e != hipSuccess) {
            if (g->d_rtab) (void)hipFree(g->d_rtab);
            if (g->d_rtab_n) (void)hipFree(g->d_rtab_n);
            g->d_rtab = nullptr;
            g->d_rtab_n = nullptr;
            return device_fail(e, "record table");
        }
        g->rtab_bytes = (int64_t)(rb + nb);
        replan_backprojection(g);
    }
    if (bytes) *bytes = g->rtab_bytes;
    return ok();
}

static cvp_status prepare(const cvp_geometry *g, const cvp_options *o, const void *in, void *outp,
                          cvp::DevGeom &G)
{
    if (!g) return fail(CVP_E_INVALID, "geometry is NULL");
    if (!o) return fail(CVP_E_INVALID, "options is NULL");
    if (!in) return fail(CVP_E_INVALID, "input pointer is NULL");
    if (!outp) return fail(CVP_E_INVALID, "output pointer is NULL");
    if (in == outp) return fail(CVP_E_INVALID, "input and output alias");
    if (o->variant != CVP_EXACT && o->variant != CVP_RELAXED && o->variant != CVP_TT)
        return fail(CVP_E_INVALID, "options.variant = %d", (int)o->variant);
    if (o->variant == CVP_TT && (o->scaling != CVP_SCALE_COS || o->elevation_correction != 0 || o->flags != 0))
        return fail(CVP_E_INVALID, "options: the TT projector estimates the area-averaged line integral and takes "
                                   "scaling CVP_SCALE_COS, elevation_correction 0 and no flags");
    if (o->elevation_correction != 0 && o->elevation_correction != 1)
        return fail(CVP_E_INVALID, "options.elevation_correction = %d", o->elevation_correction);
    if (o->scaling != CVP_SCALE_SOLID_ANGLE && o->scaling != CVP_SCALE_COS && o->scaling != CVP_SCALE_NONE)
        return fail(CVP_E_INVALID, "options.scaling = %d", (int)o->scaling);
    if (o->flags & ~CVP_FLAG_RAW_VOLUME) return fail(CVP_E_INVALID, "options.flags = 0x%x", o->flags);
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return device_fail(e, "hipGetDevice");
    if (dev != g->device)
        return fail(CVP_E_INVALID, "geometry lives on device %d but device %d is current", g->device, dev);
    G = g->base;
    G.sigma = o->scaling == CVP_SCALE_NONE ? nullptr : g->d_sigma[o->scaling == CVP_SCALE_COS ? 1 : 0];
    G.raw_volume = (o->flags & CVP_FLAG_RAW_VOLUME) ? 1 : 0;
    if (o->variant == CVP_TT) {
        // no pixel factor; the fixed-point bounds of footprint weights
        G.sigma = nullptr;
        G.wone_bound = g->wone_tt;
        G.wsum_bound = g->wsum_tt;
    } else if (g->d_rtab) {
        // the cached piece records (the same bits the kernels would compute)
        G.rtab = g->d_rtab;
        G.rtab_n = g->d_rtab_n;
        G.rtab_pmax = g->pmax;
    }
    return CVP_OK;
}

cvp_status cvp_project(const cvp_geometry *g, const cvp_options *o, const float *d_vol,
                       float *d_proj, void *stream)
{
    cvp::DevGeom G;
    cvp_status st = prepare(g, o, d_vol, d_proj, G);
    if (st != CVP_OK) return st;
    hipError_t e = cvp::launch_project(G, g->pl, model_of(o), o->elevation_correction != 0,
                                       d_vol, d_proj, nullptr, (hipStream_t)stream);
    if (e != hipSuccess) return device_fail(e, "projection launch");
    return ok();
}

cvp_status cvp_project_workspace_size(const cvp_geometry *g, int64_t *bytes)
{
    if (!g) return fail(CVP_E_INVALID, "geometry is NULL");
    if (!bytes) return fail(CVP_E_INVALID, "bytes is NULL");
    *bytes = cvp::group_max_cells(g->base) * (int64_t)sizeof(unsigned);
    return ok();
}

cvp_status cvp_project_ws(const cvp_geometry *g, const cvp_options *o, const float *d_vol, float *d_proj,
                          void *d_work, int64_t work_bytes, void *stream)
{
    cvp::DevGeom G;
    cvp_status st = prepare(g, o, d_vol, d_proj, G);
    if (st != CVP_OK) return st;
    if (!d_work) return fail(CVP_E_INVALID, "work is NULL");
    const int64_t need = cvp::group_max_cells(g->base) * (int64_t)sizeof(unsigned);
    if (work_bytes < need)
        return fail(CVP_E_INVALID, "work_bytes = %lld, need %lld (cvp_project_workspace_size)", (long long)work_bytes,
                    (long long)need);
    if (reinterpret_cast<uintptr_t>(d_work) & 3) return fail(CVP_E_INVALID, "work must be 4-byte aligned");
    if (d_work == (const void *)d_vol || d_work == (void *)d_proj)
        return fail(CVP_E_INVALID, "work aliases the volume or the projections");
    hipError_t e = cvp::launch_project(G, g->pl, model_of(o), o->elevation_correction != 0,
                                       d_vol, d_proj, (unsigned *)d_work, (hipStream_t)stream);
    if (e != hipSuccess) return device_fail(e, "projection launch");
    return ok();
}

cvp_status cvp_project_noalloc(const cvp_geometry *g, const cvp_options *o, const float *d_vol, float *d_proj,
                               void *stream)
{
    cvp::DevGeom G;
    cvp_status st = prepare(g, o, d_vol, d_proj, G);
    if (st != CVP_OK) return st;
    const int64_t need = cvp::group_max_cells(g->base);
    if (need > cvp::kStaticScratchWords)
        return fail(CVP_E_UNSUPPORTED,
                    "n2 * ceil(n1 / 16) = %lld exceeds the fixed scratch of %lld words (CVP_NOALLOC_MAX_GROUPS)",
                    (long long)need, (long long)cvp::kStaticScratchWords);
    unsigned *work = nullptr;
    hipError_t e = cvp::static_scratch(&work);
    if (e != hipSuccess) return device_fail(e, "scratch symbol address");
    e = cvp::launch_project(G, g->pl, model_of(o), o->elevation_correction != 0, d_vol, d_proj, work,
                            (hipStream_t)stream);
    if (e != hipSuccess) return device_fail(e, "projection launch");
    return ok();
}

cvp_status cvp_project_siddon(const cvp_geometry *g, int32_t K, const float *d_vol, float *d_proj, void *stream)
{
    if (K < 1 || K > 1024) return fail(CVP_E_INVALID, "K = %d (must be 1..1024)", K);
    const cvp_options o{CVP_EXACT, 0, CVP_SCALE_NONE, 0u};
    cvp::DevGeom G;
    cvp_status st = prepare(g, &o, d_vol, d_proj, G);
    if (st != CVP_OK) return st;
    hipError_t e = cvp::launch_siddon(G, K, d_vol, d_proj, (hipStream_t)stream);
    if (e != hipSuccess) return device_fail(e, "SiddonK launch");
    return ok();
}

cvp_status cvp_backproject(const cvp_geometry *g, const cvp_options *o, const float *d_proj,
                           float *d_vol, void *stream)
{
    cvp::DevGeom G;
    cvp_status st = prepare(g, o, d_proj, d_vol, G);
    if (st != CVP_OK) return st;
    hipError_t e = cvp::launch_backproject(G, back_plan(g, G), model_of(o), o->elevation_correction != 0,
                                           d_proj, d_vol, (hipStream_t)stream);
    if (e != hipSuccess) return device_fail(e, "backprojection launch");
    return ok();
}

// Views v0, v0 + stride, ..., v0 + (count - 1) stride of a geometry: the
// view table and the projection pointer start at v0 and step by stride.
static cvp_status view_subset(const cvp_geometry *g, int32_t view0, int32_t stride, int32_t count,
                              cvp::DevGeom &G, int64_t &proj_offset)
{
    const int V = g->base.nviews;
    if (view0 < 0 || view0 >= V) return fail(CVP_E_INVALID, "view0 = %d (must be 0..%d)", view0, V - 1);
    if (stride < 1) return fail(CVP_E_INVALID, "view_stride = %d (must be >= 1)", stride);
    if (count < 1 || (int64_t)view0 + (int64_t)(count - 1) * stride >= V)
        return fail(CVP_E_INVALID, "n_views = %d: views %d + k * %d run past the last view (%d)", count, view0,
                    stride, V - 1);
    G.views = g->d_views + view0;
    G.vstride = stride;
    G.nviews = count;
    proj_offset = (int64_t)view0 * G.N * G.M;
    if (G.sigma && G.sigma_views) G.sigma += proj_offset;
    if (G.rtab) {
        const int64_t cols = (int64_t)view0 * G.n2 * G.n1;
        G.rtab += cols * G.rtab_pmax * cvp::kRecFloats;
        G.rtab_n += cols;
    }
    return CVP_OK;
}

cvp_status cvp_project_views(const cvp_geometry *g, const cvp_options *o, const float *d_vol, float *d_proj,
                             int32_t view0, int32_t view_stride, int32_t n_views, void *d_work, int64_t work_bytes,
                             void *stream)
{
    cvp::DevGeom G;
    cvp_status st = prepare(g, o, d_vol, d_proj, G);
    if (st != CVP_OK) return st;
    int64_t off = 0;
    st = view_subset(g, view0, view_stride, n_views, G, off);
    if (st != CVP_OK) return st;
    if (d_work) {
        const int64_t need = cvp::group_max_cells(g->base) * (int64_t)sizeof(unsigned);
        if (work_bytes < need)
            return fail(CVP_E_INVALID, "work_bytes = %lld, need %lld (cvp_project_workspace_size)",
                        (long long)work_bytes, (long long)need);
        if (reinterpret_cast<uintptr_t>(d_work) & 3) return fail(CVP_E_INVALID, "work must be 4-byte aligned");
    }
    cvp::ProjLaunch pl{};
    if (!cvp::plan_projection(G.N, G.n2, G.M, n_views, g->pmax, g->pl.U, pl))
        return fail(CVP_E_UNSUPPORTED, "projection plan");
    hipError_t e = cvp::launch_project(G, pl, model_of(o), o->elevation_correction != 0, d_vol,
                                       d_proj + off, (unsigned *)d_work, (hipStream_t)stream);
    if (e != hipSuccess) return device_fail(e, "projection launch");
    return ok();
}

cvp_status cvp_backproject_views(const cvp_geometry *g, const cvp_options *o, const float *d_proj, float *d_vol,
                                 int32_t view0, int32_t view_stride, int32_t n_views, void *stream)
{
    cvp::DevGeom G;
    cvp_status st = prepare(g, o, d_proj, d_vol, G);
    if (st != CVP_OK) return st;
    int64_t off = 0;
    st = view_subset(g, view0, view_stride, n_views, G, off);
    if (st != CVP_OK) return st;
    hipError_t e = cvp::launch_backproject(G, back_plan(g, G), model_of(o), o->elevation_correction != 0,
                                           d_proj + off, d_vol, (hipStream_t)stream);
    if (e != hipSuccess) return device_fail(e, "backprojection launch");
    return ok();
}

}  // extern "C"

struct cvp_batch {
    int n = 0;
    int device = 0;
    std::vector<const cvp_geometry *> geoms;
    cvp::BatchProblem *d_probs = nullptr;
    cvp::BatchTable *d_ptab = nullptr;
    // backprojection groups g = 3 p + w: piece stride 4 (p = 0) or 8 (p = 1),
    // stack width 16, 8, 4 (w = 0, 1, 2)
    cvp::BatchTable *d_btab[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    int *d_counter = nullptr;         // [0] projection, [1 + g] backprojection group g
    std::vector<unsigned *> d_gmax;   // per problem: per-group maxima of the volume
    size_t plds = 0, blds[6] = {0, 0, 0, 0, 0, 0};
    int pgrid = 0, bgrid[6] = {0, 0, 0, 0, 0, 0};
    bool cached = false;                  // every member reads its geometry's cached records
    std::vector<const float *> rtabs;     // the tables captured at creation
};

extern "C" {

void cvp_batch_destroy(cvp_batch *b)
{
    if (!b) return;
    if (b->d_probs) (void)hipFree(b->d_probs);
    if (b->d_ptab) (void)hipFree(b->d_ptab);
    for (cvp::BatchTable *t : b->d_btab)
        if (t) (void)hipFree(t);
    if (b->d_counter) (void)hipFree(b->d_counter);
    for (unsigned *t : b->d_gmax)
        if (t) (void)hipFree(t);
    delete b;
}

cvp_status cvp_batch_create(const cvp_geometry *const *geoms, int32_t n, cvp_batch **out)
{
    if (!out) return fail(CVP_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!geoms) return fail(CVP_E_INVALID, "geoms is NULL");
    if (n < 1 || n > cvp::kMaxBatch) return fail(CVP_E_INVALID, "n = %d (must be 1..%d)", n, cvp::kMaxBatch);
    for (int q = 0; q < n; ++q) {
        if (!geoms[q]) return fail(CVP_E_INVALID, "geoms[%d] is NULL", q);
        if (geoms[q]->device != geoms[0]->device)
            return fail(CVP_E_INVALID, "geoms[%d] lives on another device", q);
        if (geoms[q]->bl.pmax > 8)
            return fail(CVP_E_UNSUPPORTED, "geoms[%d]: voxels project onto more than 8 detector columns "
                                           "(batched kernels keep at most 8 pieces per column)", q);
    }
    cvp_batch *b = new (std::nothrow) cvp_batch();
    if (!b) return fail(CVP_E_NOMEM, "host allocation");
    b->n = n;
    b->device = geoms[0]->device;
    b->geoms.assign(geoms, geoms + n);
    // with every member's records cached the batched kernels read them too
    b->cached = true;
    for (int q = 0; q < n; ++q) b->cached = b->cached && geoms[q]->d_rtab != nullptr;
    // Projection: every problem keeps its own plan (the batched kernel
    // dispatches on the piece stride per item), so its results are those of
    // its own launches.  Backprojection: every problem keeps its own piece
    // stride and stack width, and the batch runs one persistent launch per
    // (stride, width) present; backprojection sums do not depend on the plan,
    // so the results still equal single launches bitwise.  One dynamic LDS
    // size fits all items of a launch.
    static const int kGw[3] = {16, 8, 4};
    std::vector<cvp::BackLaunch> bls(n);
    std::vector<int> grp(n);
    for (int q = 0; q < n; ++q) {
        // the member's own stack width, else the next narrower one whose
        // 8-piece records fit
        bool planned = false;
        const int pm = geoms[q]->pmax <= 4 ? 4 : 8;
        for (int gi = 0; gi < 3 && !planned; ++gi) {
            if (kGw[gi] > geoms[q]->bl.gw) continue;
            planned = cvp::plan_backprojection(geoms[q]->base, pm, geoms[q]->zabs, geoms[q]->Dmin, kGw[gi], 0, bls[q],
                                               b->cached, cvp::kBatchStaticLds, geoms[q]->bp_wpc);
            grp[q] = (pm == 4 ? 0 : 3) + gi;
        }
        if (!planned) {
            delete b;
            return fail(CVP_E_UNSUPPORTED, "geoms[%d]: batched backprojection plan does not fit LDS", q);
        }
    }
    std::vector<cvp::BatchProblem> probs(n);
    std::vector<double> pcost(n), bcost(n);
    for (int q = 0; q < n; ++q) {
        const cvp_geometry *g = geoms[q];
        const cvp::ProjLaunch &pl = g->pl;
        const cvp::BackLaunch &bl = bls[q];
        cvp::BatchProblem &P = probs[q];
        P.G = g->base;
        P.U = pl.U;
        P.pmax = pl.pmax;
        P.gw = bl.gw;
        P.kp = bl.kp;
        P.win_cap = bl.win_cap;
        P.pitems = pl.items;
        P.ngroups = bl.ngroups;
        P.nkchunks = bl.nkchunks;
        P.bitems = bl.items;
        P.in = nullptr;
        P.out = nullptr;
        P.gmax = nullptr;   // set below
        P.stop = nullptr;   // set per call
        if (b->cached) {
            P.G.rtab = g->d_rtab;
            P.G.rtab_n = g->d_rtab_n;
            P.G.rtab_pmax = g->pmax;
            b->rtabs.push_back(g->d_rtab);
        }
        b->plds = std::max(b->plds, pl.lds);
        b->blds[grp[q]] = std::max(b->blds[grp[q]], bl.lds);
        pcost[q] = (double)g->nvox / pl.nbands;           // voxels per band (all k)
        bcost[q] = (double)g->base.nviews;                // views per voxel stack
    }
    // work segments of the members in `sel`, largest items first
    auto table = [&](const std::vector<double> &cost, bool back, int sel) {
        cvp::BatchTable T{};
        std::vector<int> ord;
        for (int q = 0; q < n; ++q)
            if (sel < 0 || grp[q] == sel) ord.push_back(q);
        std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return cost[x] > cost[y]; });
        T.n = (int)ord.size();
        T.start[0] = 0;
        for (int q = 0; q < T.n; ++q) {
            T.order[q] = ord[q];
            T.start[q + 1] = T.start[q] + (back ? probs[ord[q]].bitems : probs[ord[q]].pitems);
        }
        return T;
    };
    const cvp::BatchTable pt = table(pcost, false, -1);
    int cus = 0;
    hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device);
    if (e == hipSuccess) e = hipMalloc((void **)&b->d_probs, n * sizeof(cvp::BatchProblem));
    if (e == hipSuccess) e = hipMalloc((void **)&b->d_ptab, sizeof(cvp::BatchTable));
    if (e == hipSuccess) e = hipMalloc((void **)&b->d_counter, 7 * sizeof(int));
    for (int gi = 0; gi < 6 && e == hipSuccess; ++gi) {
        if (b->blds[gi] == 0) continue;   // no member with this stride and width
        const cvp::BatchTable bt = table(bcost, true, gi);
        e = hipMalloc((void **)&b->d_btab[gi], sizeof(cvp::BatchTable));
        if (e == hipSuccess) e = hipMemcpy(b->d_btab[gi], &bt, sizeof(bt), hipMemcpyHostToDevice);
        b->bgrid[gi] = cus * cvp::batched_blocks_per_cu(true, b->blds[gi], kGw[gi % 3], gi < 3 ? 4 : 8, b->cached);
    }
    b->d_gmax.assign(n, nullptr);
    for (int q = 0; q < n && e == hipSuccess; ++q) {
        e = hipMalloc((void **)&b->d_gmax[q], cvp::group_max_cells(probs[q].G) * sizeof(unsigned));
        probs[q].gmax = b->d_gmax[q];
    }
    if (e == hipSuccess) e = hipMemcpy(b->d_probs, probs.data(), n * sizeof(cvp::BatchProblem), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b->d_ptab, &pt, sizeof(pt), hipMemcpyHostToDevice);
    if (e != hipSuccess) { cvp_batch_destroy(b); return device_fail(e, "batch tables"); }
    b->pgrid = cus * cvp::batched_blocks_per_cu(false, b->plds, 16, 8, b->cached);
    *out = b;
    return ok();
}

static cvp_status batched(const cvp_batch *b, const cvp_options *o, const float *const *ins,
                          float *const *outs, void *stream, bool backward, const double *const *stops = nullptr)
{
    if (!b) return fail(CVP_E_INVALID, "batch is NULL");
    if (!o) return fail(CVP_E_INVALID, "options is NULL");
    if (!ins || !outs) return fail(CVP_E_INVALID, "pointer array is NULL");
    if (o->variant == CVP_TT) return fail(CVP_E_UNSUPPORTED, "the batched launches run the cutting voxel projector only");
    if (b->cached)
        for (int q = 0; q < b->n; ++q)
            if (b->geoms[q]->d_rtab != b->rtabs[q])
                return fail(CVP_E_INVALID, "problem %d: its record table changed since cvp_batch_create "
                                           "(keep the tables while the batch lives)", q);
    cvp::BatchIO io{};
    io.n = b->n;
    io.raw = (o->flags & CVP_FLAG_RAW_VOLUME) ? 1 : 0;
    for (int q = 0; q < b->n; ++q) {
        cvp::DevGeom G;
        cvp_status st = prepare(b->geoms[q], o, ins[q], outs[q], G);
        if (st != CVP_OK) return fail(st, "problem %d: %s", q, g_err.c_str());
        io.in[q] = ins[q];
        io.out[q] = outs[q];
        io.sigma[q] = G.sigma;
        io.stop[q] = stops ? stops[q] : nullptr;
    }
    if (!backward) {
        // per-group maxima of every volume, for the projection items' scales
        for (int q = 0; q < b->n; ++q) {
            hipError_t e = cvp::launch_group_max(b->geoms[q]->base, ins[q], b->d_gmax[q], (hipStream_t)stream,
                                                 io.stop[q]);
            if (e != hipSuccess) return device_fail(e, "batched group maxima");
        }
    }
    const bool ex = o->variant == CVP_EXACT, ec = o->elevation_correction != 0;
    hipError_t e = hipSuccess;
    if (!backward) {
        e = cvp::launch_batched(false, b->d_probs, b->d_ptab, b->d_counter, io, ex, ec, b->pgrid, b->plds, 16, 8,
                                b->cached, (hipStream_t)stream);
    } else {
        static const int kGw[3] = {16, 8, 4};
        for (int gi = 0; gi < 6 && e == hipSuccess; ++gi)
            if (b->d_btab[gi])
                e = cvp::launch_batched(true, b->d_probs, b->d_btab[gi], b->d_counter + 1 + gi, io, ex, ec,
                                        b->bgrid[gi], b->blds[gi], kGw[gi % 3], gi < 3 ? 4 : 8, b->cached,
                                        (hipStream_t)stream);
    }
    if (e != hipSuccess) return device_fail(e, "batched launch");
    return ok();
}

cvp_status cvp_project_batched(const cvp_batch *b, const cvp_options *o, const float *const *d_vols,
                               float *const *d_projs, void *stream)
{
    return batched(b, o, d_vols, d_projs, stream, false);
}

cvp_status cvp_backproject_batched(const cvp_batch *b, const cvp_options *o, const float *const *d_projs,
                                   float *const *d_vols, void *stream)
{
    return batched(b, o, d_projs, d_vols, stream, true);
}

cvp_status cvp_cgls_workspace_size(int64_t n_voxels, int64_t n_pixels_total, int64_t *bytes)
{
    if (!bytes) return fail(CVP_E_INVALID, "bytes is NULL");
    if (n_voxels < 0 || n_pixels_total < 0) return fail(CVP_E_INVALID, "negative size");
    *bytes = cvp::kCglsWorkDoubles * (int64_t)sizeof(double);
    return ok();
}

static cvp_status cgls_args(const cvp_geometry *g, const cvp_options *o, const void *x,
                            const void *r, const void *s, const void *p, const void *q,
                            const void *work, cvp::DevGeom &G)
{
    const void *ptrs[6] = {x, r, s, p, q, work};
    const char *names[6] = {"x", "r", "s", "p", "q", "work"};
    for (int a = 0; a < 6; ++a)
        if (!ptrs[a]) return fail(CVP_E_INVALID, "%s is NULL", names[a]);
    for (int a = 0; a < 5; ++a)
        for (int b = a + 1; b < 5; ++b)
            if (ptrs[a] == ptrs[b]) return fail(CVP_E_INVALID, "%s and %s alias", names[a], names[b]);
    if (reinterpret_cast<uintptr_t>(work) & 7) return fail(CVP_E_INVALID, "work must be 8-byte aligned");
    return prepare(g, o, x, const_cast<void *>(r), G);
}

cvp_status cvp_cgls_start(const cvp_geometry *g, const cvp_options *o, const float *d_b, float *d_x,
                          float *d_r, float *d_s, float *d_p, float *d_q, void *d_work, void *stream)
{
    cvp::DevGeom G;
    if (!d_b) return fail(CVP_E_INVALID, "b is NULL");
    cvp_status st = cgls_args(g, o, d_x, d_r, d_s, d_p, d_q, d_work, G);
    if (st != CVP_OK) return st;
    hipStream_t sm = (hipStream_t)stream;
    double *sc = (double *)d_work;
    double *part = sc + cvp::kCglsScalars + 2 * cvp::kCglsHistory;
    const int ex = model_of(o);
    const bool ec = o->elevation_correction != 0;
    // s (volume sized) is free until A^T r: it holds the projection's
    // per-group maxima
    hipError_t e = cvp::launch_project(G, g->pl, ex, ec, d_x, d_q, (unsigned *)d_s, sm);
    if (e == hipSuccess) e = cvp::blas_residual(d_r, d_b, d_q, g->npix, sm);
    if (e == hipSuccess) e = cvp::launch_backproject(G, back_plan(g, G), ex, ec, d_r, d_s, sm);
    if (e == hipSuccess) e = cvp::blas_update_p(d_p, d_s, g->nvox, sc, 1, sm);
    if (e == hipSuccess) e = cvp::blas_dot(d_s, d_s, g->nvox, part, sc, 0, nullptr, sm);
    if (e != hipSuccess) return device_fail(e, "cgls start");
    return ok();
}

cvp_status cvp_cgls_iterate(const cvp_geometry *g, const cvp_options *o, int32_t n_iter, float *d_x,
                            float *d_r, float *d_s, float *d_p, float *d_q, void *d_work, void *stream)
{
    cvp::DevGeom G;
    if (n_iter < 0) return fail(CVP_E_INVALID, "n_iter = %d", n_iter);
    cvp_status st = cgls_args(g, o, d_x, d_r, d_s, d_p, d_q, d_work, G);
    if (st != CVP_OK) return st;
    hipStream_t sm = (hipStream_t)stream;
    double *sc = (double *)d_work;
    double *part = sc + cvp::kCglsScalars + 2 * cvp::kCglsHistory;
    const int ex = model_of(o);
    const bool ec = o->elevation_correction != 0;
    // every kernel of an iteration returns at once once the stop flag is up
    const double *stop = sc + cvp::kCglsStop;
    hipError_t e = hipSuccess;
    for (int it = 0; it < n_iter && e == hipSuccess; ++it) {
        e = cvp::launch_project(G, g->pl, ex, ec, d_p, d_q, (unsigned *)d_s, sm, stop);       // q = A p (s free)
        if (e == hipSuccess) e = cvp::blas_dot(d_q, d_q, g->npix, part, sc, 1, nullptr, sm, stop);   // alpha
        if (e == hipSuccess) e = cvp::blas_update_xr(d_x, d_p, g->nvox, d_r, d_q, g->npix, sc, part, sm, stop);
        if (e == hipSuccess) e = cvp::launch_backproject(G, back_plan(g, G), ex, ec, d_r, d_s, sm, stop);   // s = A^T r
        if (e == hipSuccess) e = cvp::blas_dot(d_s, d_s, g->nvox, part, sc, 2, nullptr, sm, stop);   // beta
        if (e == hipSuccess) e = cvp::blas_update_p(d_p, d_s, g->nvox, sc, 0, sm, stop);           // p
    }
    if (e != hipSuccess) return device_fail(e, "cgls iterate");
    return ok();
}

// Batched CGLS: the single-problem recurrences per problem, each operator
// step one batched launch over all problems.
struct BatchedCgls {
    const float *const *b;
    float *const *x, *const *r, *const *s, *const *p, *const *q;
    void *const *work;
};

static cvp_status cgls_batched_args(const cvp_batch *bt, const cvp_options *o, const BatchedCgls &V,
                                    bool need_b)
{
    if (!bt) return fail(CVP_E_INVALID, "batch is NULL");
    if (!V.x || !V.r || !V.s || !V.p || !V.q || !V.work || (need_b && !V.b))
        return fail(CVP_E_INVALID, "pointer array is NULL");
    for (int k = 0; k < bt->n; ++k) {
        if (need_b && !V.b[k]) return fail(CVP_E_INVALID, "problem %d: b is NULL", k);
        cvp::DevGeom G;
        cvp_status st = cgls_args(bt->geoms[k], o, V.x[k], V.r[k], V.s[k], V.p[k], V.q[k], V.work[k], G);
        if (st != CVP_OK) return fail(st, "problem %d: %s", k, g_err.c_str());
    }
    // no vector or workspace may serve two problems
    std::vector<const void *> all;
    for (int k = 0; k < bt->n; ++k)
        for (const void *ptr : {(const void *)V.x[k], (const void *)V.r[k], (const void *)V.s[k],
                                (const void *)V.p[k], (const void *)V.q[k], (const void *)V.work[k]})
            all.push_back(ptr);
    std::sort(all.begin(), all.end());
    if (std::adjacent_find(all.begin(), all.end()) != all.end())
        return fail(CVP_E_INVALID, "a vector or workspace is shared between problems");
    return CVP_OK;
}

static double *cgls_scalars(void *work) { return (double *)work; }
static double *cgls_partials(void *work) { return (double *)work + cvp::kCglsScalars + 2 * cvp::kCglsHistory; }

cvp_status cvp_cgls_batched_start(const cvp_batch *bt, const cvp_options *o, const float *const *d_b,
                                  float *const *d_x, float *const *d_r, float *const *d_s,
                                  float *const *d_p, float *const *d_q, void *const *d_work, void *stream)
{
    const BatchedCgls V{d_b, d_x, d_r, d_s, d_p, d_q, d_work};
    cvp_status st = cgls_batched_args(bt, o, V, true);
    if (st != CVP_OK) return st;
    hipStream_t sm = (hipStream_t)stream;
    const int n = bt->n;
    st = batched(bt, o, (const float *const *)d_x, d_q, stream, false);             // q = A x
    if (st != CVP_OK) return st;
    hipError_t e = hipSuccess;
    for (int k = 0; k < n && e == hipSuccess; ++k)
        e = cvp::blas_residual(d_r[k], d_b[k], d_q[k], bt->geoms[k]->npix, sm);     // r = b - q
    if (e != hipSuccess) return device_fail(e, "batched cgls start");
    st = batched(bt, o, (const float *const *)d_r, d_s, stream, true);              // s = A^T r
    if (st != CVP_OK) return st;
    for (int k = 0; k < n && e == hipSuccess; ++k) {
        const int64_t nv = bt->geoms[k]->nvox;
        e = cvp::blas_update_p(d_p[k], d_s[k], nv, cgls_scalars(d_work[k]), 1, sm);
        if (e == hipSuccess)
            e = cvp::blas_dot(d_s[k], d_s[k], nv, cgls_partials(d_work[k]), cgls_scalars(d_work[k]), 0, nullptr, sm);
    }
    if (e != hipSuccess) return device_fail(e, "batched cgls start");
    return ok();
}

cvp_status cvp_cgls_batched_iterate(const cvp_batch *bt, const cvp_options *o, int32_t n_iter,
                                    float *const *d_x, float *const *d_r, float *const *d_s,
                                    float *const *d_p, float *const *d_q, void *const *d_work, void *stream)
{
    if (n_iter < 0) return fail(CVP_E_INVALID, "n_iter = %d", n_iter);
    const BatchedCgls V{nullptr, d_x, d_r, d_s, d_p, d_q, d_work};
    cvp_status st = cgls_batched_args(bt, o, V, false);
    if (st != CVP_OK) return st;
    hipStream_t sm = (hipStream_t)stream;
    const int n = bt->n;
    // each problem's kernels and work items are skipped once its stop flag is up
    const double *stops[cvp::kMaxBatch];
    for (int k = 0; k < n; ++k) stops[k] = cgls_scalars(d_work[k]) + cvp::kCglsStop;
    hipError_t e = hipSuccess;
    for (int it = 0; it < n_iter; ++it) {
        st = batched(bt, o, (const float *const *)d_p, d_q, stream, false, stops);  // q = A p
        if (st != CVP_OK) return st;
        for (int k = 0; k < n && e == hipSuccess; ++k) {
            const cvp_geometry *g = bt->geoms[k];
            double *sc = cgls_scalars(d_work[k]), *part = cgls_partials(d_work[k]);
            e = cvp::blas_dot(d_q[k], d_q[k], g->npix, part, sc, 1, nullptr, sm, stops[k]);   // alpha
            if (e == hipSuccess)
                e = cvp::blas_update_xr(d_x[k], d_p[k], g->nvox, d_r[k], d_q[k], g->npix, sc, part, sm, stops[k]);
        }
        if (e != hipSuccess) break;
        st = batched(bt, o, (const float *const *)d_r, d_s, stream, true, stops);   // s = A^T r
        if (st != CVP_OK) return st;
        for (int k = 0; k < n && e == hipSuccess; ++k) {
            const int64_t nv = bt->geoms[k]->nvox;
            double *sc = cgls_scalars(d_work[k]), *part = cgls_partials(d_work[k]);
            e = cvp::blas_dot(d_s[k], d_s[k], nv, part, sc, 2, nullptr, sm, stops[k]);        // beta
            if (e == hipSuccess) e = cvp::blas_update_p(d_p[k], d_s[k], nv, sc, 0, sm, stops[k]);   // p
        }
        if (e != hipSuccess) break;
    }
    if (e != hipSuccess) return device_fail(e, "batched cgls iterate");
    return ok();
}

// ------------------------------------------------------------------ OS-SART

static int subset_count(int V, int T, int t) { return (V - t + T - 1) / T; }

cvp_status cvp_sart_setup(const cvp_geometry *g, const cvp_options *o, int32_t n_subsets, float *d_rowsum,
                          float *d_colsum, float *d_q, void *stream)
{
    cvp::DevGeom G;
    if (!d_colsum || !d_q) return fail(CVP_E_INVALID, "colsum or q is NULL");
    cvp_status st = prepare(g, o, d_colsum, d_rowsum, G);
    if (st != CVP_OK) return st;
    const int V = G.nviews;
    if (n_subsets < 1 || n_subsets > V) return fail(CVP_E_INVALID, "n_subsets = %d (must be 1..%d)", n_subsets, V);
    if (d_q == d_rowsum) return fail(CVP_E_INVALID, "q and rowsum alias");
    hipStream_t sm = (hipStream_t)stream;
    const int ex = model_of(o);
    const bool ec = o->elevation_correction != 0;
    // R = A 1 (all views), C_t = A_t^T 1 (views t, t + T, ...)
    hipError_t e = cvp::blas_fill(d_colsum, g->nvox, 1.0f, sm);
    if (e == hipSuccess) e = cvp::launch_project(G, g->pl, ex, ec, d_colsum, d_rowsum, nullptr, sm);
    if (e == hipSuccess) e = cvp::blas_fill(d_q, g->npix, 1.0f, sm);
    for (int t = 0; t < n_subsets && e == hipSuccess; ++t) {
        cvp::DevGeom Gt = G;
        int64_t off = 0;
        view_subset(g, t, n_subsets, subset_count(V, n_subsets, t), Gt, off);
        e = cvp::launch_backproject(Gt, back_plan(g, Gt), ex, ec, d_q + off, d_colsum + (size_t)t * g->nvox, sm);
    }
    if (e != hipSuccess) return device_fail(e, "sart setup");
    return ok();
}

cvp_status cvp_sart_iterate(const cvp_geometry *g, const cvp_options *o, int32_t n_subsets, int32_t n_sweeps,
                            float lambda, int32_t nonneg, const float *d_b, float *d_x, const float *d_rowsum,
                            const float *d_colsum, float *d_q, float *d_z, void *stream)
{
    cvp::DevGeom G;
    if (!d_b || !d_rowsum || !d_colsum || !d_q || !d_z) return fail(CVP_E_INVALID, "NULL pointer");
    cvp_status st = prepare(g, o, d_b, d_x, G);
    if (st != CVP_OK) return st;
    const int V = G.nviews;
    if (n_subsets < 1 || n_subsets > V) return fail(CVP_E_INVALID, "n_subsets = %d (must be 1..%d)", n_subsets, V);
    if (n_sweeps < 0) return fail(CVP_E_INVALID, "n_sweeps = %d", n_sweeps);
    if (!std::isfinite(lambda) || !(lambda > 0.0f)) return fail(CVP_E_INVALID, "lambda must be finite and > 0");
    if (d_q == d_b || d_q == d_rowsum || d_z == d_x || (const float *)d_z == d_colsum)
        return fail(CVP_E_INVALID, "work vectors alias inputs");
    hipStream_t sm = (hipStream_t)stream;
    const int ex = model_of(o);
    const bool ec = o->elevation_correction != 0;
    const int64_t nm = (int64_t)G.N * G.M;
    hipError_t e = hipSuccess;
    for (int it = 0; it < n_sweeps && e == hipSuccess; ++it) {
        for (int t = 0; t < n_subsets && e == hipSuccess; ++t) {
            cvp::DevGeom Gt = G;
            int64_t off = 0;
            const int cnt = subset_count(V, n_subsets, t);
            view_subset(g, t, n_subsets, cnt, Gt, off);
            cvp::ProjLaunch pl{};
            cvp::plan_projection(G.N, G.n2, G.M, cnt, g->pmax, g->pl.U, pl);
            // q_t = A_t x (z is free: it holds the per-group maxima)
            e = cvp::launch_project(Gt, pl, ex, ec, d_x, d_q + off, (unsigned *)d_z, sm);
            if (e == hipSuccess)
                e = cvp::sart_residual_views(d_q + off, d_b + off, d_rowsum + off, nm, cnt, nm * n_subsets, sm);
            if (e == hipSuccess) e = cvp::launch_backproject(Gt, back_plan(g, Gt), ex, ec, d_q + off, d_z, sm);
            if (e == hipSuccess)
                e = cvp::sart_update_x(d_x, d_z, d_colsum + (size_t)t * g->nvox, g->nvox, lambda, nonneg != 0, sm);
        }
    }
    if (e != hipSuccess) return device_fail(e, "sart iterate");
    return ok();
}

// ------------------------------------------------------------------ LSQR

cvp_status cvp_lsqr_workspace_size(int64_t n_voxels, int64_t n_pixels_total, int64_t *bytes)
{
    if (!bytes) return fail(CVP_E_INVALID, "bytes is NULL");
    if (n_voxels < 0 || n_pixels_total < 0) return fail(CVP_E_INVALID, "negative size");
    *bytes = cvp::kLsqrWorkDoubles * (int64_t)sizeof(double);
    return ok();
}

static cvp_status lsqr_args(const cvp_geometry *g, const cvp_options *o, const void *x, const void *u,
                            const void *v, const void *w, const void *q, const void *s, const void *work,
                            cvp::DevGeom &G)
{
    const void *ptrs[7] = {x, u, v, w, q, s, work};
    const char *names[7] = {"x", "u", "v", "w", "q", "s", "work"};
    for (int a = 0; a < 7; ++a)
        if (!ptrs[a]) return fail(CVP_E_INVALID, "%s is NULL", names[a]);
    for (int a = 0; a < 7; ++a)
        for (int b = a + 1; b < 7; ++b)
            if (ptrs[a] == ptrs[b]) return fail(CVP_E_INVALID, "%s and %s alias", names[a], names[b]);
    if (reinterpret_cast<uintptr_t>(work) & 7) return fail(CVP_E_INVALID, "work must be 8-byte aligned");
    return prepare(g, o, x, const_cast<void *>(u), G);
}

cvp_status cvp_lsqr_start(const cvp_geometry *g, const cvp_options *o, const float *d_b, float *d_x, float *d_u,
                          float *d_v, float *d_w, float *d_q, float *d_s, void *d_work, void *stream)
{
    cvp::DevGeom G;
    if (!d_b) return fail(CVP_E_INVALID, "b is NULL");
    cvp_status st = lsqr_args(g, o, d_x, d_u, d_v, d_w, d_q, d_s, d_work, G);
    if (st != CVP_OK) return st;
    hipStream_t sm = (hipStream_t)stream;
    double *sc = (double *)d_work;
    const int ex = model_of(o);
    const bool ec = o->elevation_correction != 0;
    // beta u = b - A x;  alpha v = A^T u;  w = v
    hipError_t e = cvp::launch_project(G, g->pl, ex, ec, d_x, d_q, (unsigned *)d_s, sm);
    if (e == hipSuccess) e = cvp::blas_residual(d_u, d_b, d_q, g->npix, sm);
    if (e == hipSuccess) e = cvp::lsqr_norm(d_u, g->npix, sc, cvp::kLsqrFinBeta0, sm);
    if (e == hipSuccess) e = cvp::lsqr_scale(d_u, g->npix, sc, cvp::kLsqrBeta, sm);
    if (e == hipSuccess) e = cvp::launch_backproject(G, back_plan(g, G), ex, ec, d_u, d_v, sm);
    if (e == hipSuccess) e = cvp::lsqr_norm(d_v, g->nvox, sc, cvp::kLsqrFinAlpha0, sm);
    if (e == hipSuccess) e = cvp::lsqr_update_vxw(d_v, d_x, d_w, g->nvox, sc, 1, sm);
    if (e != hipSuccess) return device_fail(e, "lsqr start");
    return ok();
}

cvp_status cvp_lsqr_iterate(const cvp_geometry *g, const cvp_options *o, int32_t n_iter, float *d_x, float *d_u,
                            float *d_v, float *d_w, float *d_q, float *d_s, void *d_work, void *stream)
{
    cvp::DevGeom G;
    if (n_iter < 0) return fail(CVP_E_INVALID, "n_iter = %d", n_iter);
    cvp_status st = lsqr_args(g, o, d_x, d_u, d_v, d_w, d_q, d_s, d_work, G);
    if (st != CVP_OK) return st;
    hipStream_t sm = (hipStream_t)stream;
    double *sc = (double *)d_work;
    const int ex = model_of(o);
    const bool ec = o->elevation_correction != 0;
    hipError_t e = hipSuccess;
    for (int it = 0; it < n_iter && e == hipSuccess; ++it) {
        e = cvp::launch_project(G, g->pl, ex, ec, d_v, d_q, (unsigned *)d_s, sm);                 // q = A v
        if (e == hipSuccess) e = cvp::lsqr_axpby_norm(d_u, d_q, g->npix, sc, cvp::kLsqrAlpha, cvp::kLsqrFinBeta, sm);
        if (e == hipSuccess) e = cvp::lsqr_scale(d_u, g->npix, sc, cvp::kLsqrBeta, sm);           // u /= beta
        if (e == hipSuccess) e = cvp::launch_backproject(G, back_plan(g, G), ex, ec, d_u, d_s, sm);          // s = A^T u
        if (e == hipSuccess) e = cvp::lsqr_axpby_norm(d_v, d_s, g->nvox, sc, cvp::kLsqrBeta, cvp::kLsqrFinAlpha, sm);
        if (e == hipSuccess) e = cvp::lsqr_update_vxw(d_v, d_x, d_w, g->nvox, sc, 0, sm);       // v, x, w
    }
    if (e != hipSuccess) return device_fail(e, "lsqr iterate");
    return ok();
}

cvp_status cvp_cgls_set_tolerance(void *d_work, double rho_tol, double gamma_ref, void *stream)
{
    if (!d_work) return fail(CVP_E_INVALID, "work is NULL");
    if (reinterpret_cast<uintptr_t>(d_work) & 7) return fail(CVP_E_INVALID, "work must be 8-byte aligned");
    if (!std::isfinite(rho_tol) || rho_tol < 0.0) return fail(CVP_E_INVALID, "rho_tol must be finite and >= 0");
    if (!std::isfinite(gamma_ref) || gamma_ref < 0.0) return fail(CVP_E_INVALID, "gamma_ref must be finite and >= 0");
    hipError_t e = cvp::blas_set_tolerance((double *)d_work, rho_tol * rho_tol, gamma_ref, (hipStream_t)stream);
    if (e != hipSuccess) return device_fail(e, "cgls tolerance");
    return ok();
}

cvp_status cvp_dot(const float *d_a, const float *d_b, int64_t n, double *d_result, void *d_work,
                   void *stream)
{
    if (!d_a || !d_b || !d_result || !d_work) return fail(CVP_E_INVALID, "NULL pointer");
    if (n < 0) return fail(CVP_E_INVALID, "n < 0");
    double *sc = (double *)d_work;
    double *part = sc + cvp::kCglsScalars + 2 * cvp::kCglsHistory;
    hipError_t e = cvp::blas_dot(d_a, d_b, n, part, sc, 4, d_result, (hipStream_t)stream);
    if (e != hipSuccess) return device_fail(e, "dot");
    return ok();
}

}  // extern "C"
