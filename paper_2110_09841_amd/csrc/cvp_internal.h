// Internal declarations shared by the C-ABI host code and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace cvp {

constexpr int kWave = 64;             // CDNA wavefront
constexpr int kBlock = 256;           // threads per workgroup
constexpr int kWaves = kBlock / kWave;
constexpr int kRecFloats = 12;        // floats per cut-piece record

// Backprojection LDS per view of a record pass: GW x PMAX piece records, the
// GW piece counts and the 4 window bounds; a record pass covers
// back_views_per_pass views (64 lanes over GW columns x min(PMAX, 64 / GW)
// slots each).
constexpr int back_rec_floats(int gw, int pmax) { return gw * pmax * kRecFloats + gw + 4; }
constexpr int back_views_per_pass(int gw, int pmax) { return 64 / (gw * (pmax < 64 / gw ? pmax : 64 / gw)); }
constexpr float kYQuantumInv = 1024.0f;
constexpr int kBackPasses = 2;        // most 64-voxel passes per backprojection stack
constexpr int kPmaxWide = 64;         // pieces per column of the wide-footprint backprojection

// Projector models of launch_project / launch_backproject: the cutting voxel
// projector with r at the voxel centre or at each cut piece's centroid, and
// the TT separable-footprint projector on the same work split.
constexpr int kModelRelaxed = 0;
constexpr int kModelExact = 1;
constexpr int kModelTT = 2;

// Per-view source-centred frame (Sec. II-C) and intrinsics, FP64.  e1 and d
// have no x3 component (that is what makes chi1 independent of x3, the column
// identity of Sec. III-A); chi2 runs along -x3.  A projection matrix of the
// view is K [R | -R s] with rows of R e1, (0,0,-1), d and
// K = [[fb1, 0, c1], [0, fb2, c2], [0, 0, 1]] (Sec. III-C).
struct ViewGeom {
    double s1, s2, s3;   // source position
    double e1x, e1y;     // detector chi1 axis
    double dx, dy;       // principal ray direction
    double c1, c2;       // principal point (pixel-index units)
    double fb1, fb2;     // f / b1, f / b2
    double ifb2;         // b2 / f
};

// Everything a kernel needs about one problem.  Passed by value.
struct DevGeom {
    int n1, n2, n3;
    int M, N;            // detector columns (chi1), rows (chi2)
    int nviews;
    double a1, a2, a3;
    double x1lo, x2lo, x3lo;   // lower corner of the volume box
    double b1, b2, c1, c2, f;
    double fb1, fb2, b2f;      // f / b1, f / b2, b2 / f
    const ViewGeom *views;     // device; view q of a launch is views[q * vstride]
    int vstride;               // view stride: a launch may cover views v0, v0 + vstride, ... (views and
                               // the projection pointer start at v0; 1 for all views)
    const float *sigma;        // device pixel factors (nullptr: 1): [N][M], or [views][N][M] if sigma_views
    int sigma_views;           // 1: one factor table per view (views with their own intrinsics)
    int raw_volume;            // weight = cut volume (no 1/r^2)
    // Bounds on any pixel's weight sum per unit |mu| (with and without the
    // 1/r^2 factor), used to scale the projection's fixed-point sums.
    double wsum_bound, wsum_bound_raw;   // a pixel's summed weight per unit |mu|
    double wone_bound, wone_bound_raw;   // one (voxel, pixel) weight per unit |mu|
    // The geometry's cached piece records (nullptr: the kernels compute
    // their own): rtab[((q n2 + j) n1 + i) pmax + s][kRecFloats] and the
    // piece counts rtab_n[(q n2 + j) n1 + i] of column (i, j) in view q of
    // the launch (q * vstride, from the launch's first view), pieces clipped
    // to the detector columns; rtab_pmax slots per column.
    const float *rtab;
    const int *rtab_n;
    int rtab_pmax;
};

struct ProjLaunch {
    int U;           // detector columns per band
    int nbands;
    int items;       // nbands * nviews
    int chunk;       // work-item slots per XCD (grid = 8 * chunk)
    int pmax;        // 4 or 8 (8 with U <= 8 for wider footprints)
    size_t lds;      // dynamic LDS bytes
};

struct BackLaunch {
    int gw;          // columns per group (16, 8 or 4)
    int ngroups;     // groups per row (ceil(n1 / gw))
    int kp;          // 64-voxel passes per stack (1 or 2)
    int nkchunks;    // ceil(n3 / (64 * kp))
    int items;
    int chunk;
    int pmax;        // 4, 8 or kPmaxWide (then gw = 4)
    int win_cap;     // floats per wave window
    size_t lds;
    int wpc;         // workgroups per CU the LDS budget was sized for
    int shared;      // 1: one detector window per workgroup (cached records only)
};

// Batched, persistent launches over up to kMaxBatch problems.
constexpr int kMaxBatch = 32;

struct BatchProblem {        // device table entry (one per problem)
    DevGeom G;
    int U;                   // projection band width
    int pitems;              // projection work items
    int pmax;                // the problem's projection piece stride (its own plan),
    int gw;                  // the batch's backprojection stack width,
    int kp;                  // passes per stack
    int win_cap;             // and per-wave window (floats)
    int ngroups;             // backprojection column groups per row
    int nkchunks;
    int bitems;              // backprojection work items
    const float *in;         // set per call by batch_setup
    float *out;
    unsigned *gmax;          // the problem's per-group maxima (owned by the batch)
    const double *stop;      // set per call: the problem's work items are skipped while *stop != 0
};

struct BatchTable {          // device: work segments, largest items first
    int n;
    int start[kMaxBatch + 1];
    int order[kMaxBatch];
};

struct BatchIO {             // per call, by value
    int n;
    int raw;
    const float *in[kMaxBatch];
    float *out[kMaxBatch];
    const float *sigma[kMaxBatch];
    const double *stop[kMaxBatch];   // per problem, or nullptr
};

// gw, pmax: the backprojection launch's stack width (16, 8 or 4) and piece
// stride (4 or 8); cached: every member reads its geometry's cached records
hipError_t launch_batched(bool backward, BatchProblem *probs, const BatchTable *tab, int *counter,
                          const BatchIO &io, bool exact, bool ec, int grid, size_t lds, int gw, int pmax, bool cached,
                          hipStream_t s);
int batched_blocks_per_cu(bool backward, size_t lds, int gw, int pmax, bool cached);
size_t project_lds_bytes(int U, int N, int n2, int pmax);
size_t backproject_lds_bytes(int gw, int pmax, int winCap);

// CGLS workspace (FP64): scalars, then the |s|^2 and |r|^2 histories, then the
// reduction partials.
// Scalars: [0] gamma [1] |q|^2 [2] alpha [3] beta [4] gamma0 [5] |r|^2 [6] k
// [7] breakdown [8] stop flag [9] gamma threshold of the stop (0: none)
// [10] tol^2 and [11] reference gamma (0: gamma0) set by cvp_cgls_set_tolerance
constexpr int kCglsScalars = 16;
constexpr int kCglsStop = 8, kCglsThr = 9, kCglsTol2 = 10, kCglsRef = 11;
constexpr int kCglsHistory = 4096;
constexpr int kCglsPartials = 1024;
constexpr int64_t kCglsWorkDoubles = kCglsScalars + 2 * kCglsHistory + kCglsPartials;

// LSQR workspace (FP64): scalars, then the |r| and |A^T r| estimate
// histories, then the reduction partials.
enum : int {
    kLsqrAlpha = 0, kLsqrBeta = 1, kLsqrRhobar = 2, kLsqrPhibar = 3, kLsqrXStep = 4, kLsqrWStep = 5,
    kLsqrK = 6, kLsqrBreak = 7, kLsqrArnorm0 = 8, kLsqrScalars = 16
};
enum : int { kLsqrFinBeta0 = 0, kLsqrFinAlpha0 = 1, kLsqrFinBeta = 2, kLsqrFinAlpha = 3 };
constexpr int64_t kLsqrWorkDoubles = kLsqrScalars + 2 * kCglsHistory + kCglsPartials;

hipError_t blas_fill(float *p, int64_t n, float val, hipStream_t s);
hipError_t sart_residual_views(float *q, const float *b, const float *R, int64_t nm, int count, int64_t view_step,
                               hipStream_t s);
hipError_t sart_update_x(float *x, const float *z, const float *C, int64_t n, float lam, int nonneg, hipStream_t s);
hipError_t lsqr_axpby_norm(float *y, const float *x, int64_t n, double *sc, int ci, int mode, hipStream_t s);
hipError_t lsqr_norm(const float *a, int64_t n, double *sc, int mode, hipStream_t s);
hipError_t lsqr_scale(float *y, int64_t n, const double *sc, int ci, hipStream_t s);
hipError_t lsqr_update_vxw(float *v, float *x, float *w, int64_t n, const double *sc, int init, hipStream_t s);
// stop: optional device flag; a kernel returns at once while *stop != 0 (a
// converged CGLS keeps its state through the rest of a captured graph).
hipError_t blas_dot(const float *a, const float *b, int64_t n, double *partials, double *sc,
                    int mode, double *out, hipStream_t s, const double *stop = nullptr);
hipError_t blas_update_xr(float *x, const float *p, int64_t nv, float *r, const float *q, int64_t np,
                          double *sc, double *partials, hipStream_t s, const double *stop = nullptr);
hipError_t blas_update_p(float *p, const float *sv, int64_t n, const double *sc, int init,
                         hipStream_t s, const double *stop = nullptr);
hipError_t blas_set_tolerance(double *sc, double tol2, double ref, hipStream_t s);
hipError_t blas_residual(float *r, const float *b, const float *q, int64_t n, hipStream_t s);

// gmax: device scratch of group_max_cells(g) words for the per-group maxima
// of |vol| (computed by the call), or nullptr (the kernel scans the wedges).
hipError_t launch_project(const DevGeom &g, const ProjLaunch &L, int model, bool ec,
                          const float *vol, float *proj, unsigned *gmax, hipStream_t stream,
                          const double *stop = nullptr);
int64_t group_max_cells(const DevGeom &g);
hipError_t launch_group_max(const DevGeom &g, const float *vol, unsigned *gmax, hipStream_t stream,
                            const double *stop = nullptr);
// Allocation-free projection: device address (on the current device) of the
// library's fixed scratch array for the per-group maxima, looked up once per
// device; kStaticScratchWords words (1 MiB).
constexpr int64_t kStaticScratchWords = int64_t(1) << 18;
hipError_t static_scratch(unsigned **out);
// SiddonK reference projector: K x K rays per pixel, exact chord lengths.
hipError_t launch_siddon(const DevGeom &g, int K, const float *vol, float *proj, hipStream_t s);
// Fills a geometry's record table (every view, every column; pmax 4 or 8).
hipError_t launch_record_table(const DevGeom &g, int pmax, float *rec, int *cnt, hipStream_t stream);
hipError_t launch_backproject(const DevGeom &g, const BackLaunch &L, int model, bool ec,
                              const float *proj, float *vol, hipStream_t stream, const double *stop = nullptr);

}  // namespace cvp
