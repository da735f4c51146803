// Internal declarations shared by the C-ABI host code and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace cvp {

constexpr int kWave = 64;             // CDNA wavefront
constexpr int kBlock = 256;           // threads per workgroup
constexpr int kWaves = kBlock / kWave;
constexpr int kRecFloats = 12;        // floats per cut-piece record
constexpr float kYQuantumInv = 1024.0f;

// Per-view source-centred frame (Sec. II-C), FP64.  e1 and d have no x3
// component on a circular orbit (that is what makes chi1 independent of x3,
// the column identity of Sec. III-A); chi2 runs along -x3.
struct ViewGeom {
    double s1, s2, s3;   // source position
    double e1x, e1y;     // detector chi1 axis
    double dx, dy;       // principal ray direction
    double pad;
};

// Everything a kernel needs about one problem.  Passed by value.
struct DevGeom {
    int n1, n2, n3;
    int M, N;            // detector columns (chi1), rows (chi2)
    int nviews;
    double a1, a2, a3;
    double x1lo, x2lo, x3lo;   // lower corner of the volume box
    double b1, b2, c1, c2, f;
    const ViewGeom *views;     // device, [nviews]
    const float *sigma;        // device, [N][M] pixel factors (nullptr: 1)
    int raw_volume;            // weight = cut volume (no 1/r^2)
};

struct ProjLaunch {
    int U;           // detector columns per band
    int nbands;
    int items;       // nbands * nviews
    int chunk;       // items per XCD slot
    int pmax;        // 4 or 8
    size_t lds;      // dynamic LDS bytes
};

struct BackLaunch {
    int gw;          // columns per group (16, 8 or 4)
    int ngroups;     // groups per row (ceil(n1 / gw))
    int nkchunks;    // ceil(n3 / 64)
    int items;
    int chunk;
    int pmax;
    int win_cap;     // floats per wave window
    size_t lds;
};

hipError_t launch_project(const DevGeom &g, const ProjLaunch &L, bool exact, bool ec,
                          const float *vol, float *proj, hipStream_t stream);
hipError_t launch_backproject(const DevGeom &g, const BackLaunch &L, bool exact, bool ec,
                              const float *proj, float *vol, hipStream_t stream);

}  // namespace cvp
