/*
 * cvp.h -- C ABI of the MI355X (gfx950) cutting voxel projector library.
 *
 * The operators are those of Kulvait & Rose, "Cutting Voxel Projector a New
 * Approach to Construct 3D Cone Beam CT Operator" (2021):
 *
 *   b = A x    (projection, Sec. I, the operator equation A x = b)
 *   x = A^T b  (backprojection, its exact adjoint, Sec. III-D)
 *
 * with  A[(view,v,u),(i,j,k)] = sigma_uv * |V^(ijk)_(uv)| / r^2 :
 *   |V^(ijk)_(uv)|  the volume of voxel (i,j,k) cut by the ray pyramid of
 *                   pixel (u,v), estimated from the column polygons and the x3
 *                   extents of Sec. III-A (eq. cutvolume), optionally with the
 *                   elevation correction of Sec. III-B;
 *   1/r^2           the cut integral of 1/r^2 taken at one point (Sec. II-F,
 *                   eq. vox): the cut centroid (exact form) or the voxel
 *                   centre (relaxed form);
 *   sigma_uv        the per-pixel factor applied after the unscaled sums
 *                   (eq. cvpsu): 1/solid angle (eq. cvpus) or
 *                   f^2/(a cos^3 theta) (eq. cvp).
 *
 * Geometry: circular trajectory about +x3, source at
 * (D cos l, D sin l, 0); flat detector at distance f from the source, chi1
 * along (-sin l, cos l, 0), chi2 along -x3 (Sec. III-A).  Pixel (u,v) covers
 * [u-1/2,u+1/2] x [v-1/2,v+1/2] in pixel-index units; u is the column (chi1),
 * v the row (chi2).
 *
 * Memory layouts (all float32, contiguous, caller-owned device memory):
 *   volume       [n3][n2][n1]          (x1 fastest)
 *   projections  [n_views][rows][cols] (u fastest)
 *
 * Conventions for every entry point:
 *   - all functions are extern "C"; none throws;
 *   - device pointers are owned by the caller and never freed by the library;
 *   - outputs are overwritten (every element written; no prior memset needed);
 *   - operator calls are asynchronous on the given HIP stream (hipStream_t
 *     passed as void*; NULL = default stream); they allocate no memory;
 *   - a geometry object is immutable after creation and may be shared across
 *     streams and threads; distinct outputs may be computed concurrently;
 *   - on error the call returns a status and leaves a message retrievable by
 *     cvp_last_error_detail() on the same thread.
 */
#ifndef CVP_H
#define CVP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CVP_OK = 0,
    CVP_E_INVALID = 1,      /* bad argument; the message names the field */
    CVP_E_NOMEM = 2,        /* host or device allocation failed */
    CVP_E_DEVICE = 3,       /* HIP runtime error (no device, launch failure) */
    CVP_E_UNSUPPORTED = 4,  /* valid but outside what the kernels handle */
    CVP_E_BREAKDOWN = 5     /* CGLS: zero search direction norm */
} cvp_status;

typedef enum {
    CVP_EXACT = 0,          /* r at the centroid of each cut piece */
    CVP_RELAXED = 1,        /* r at the voxel centre (speed-optimised form) */
    CVP_TT = 2              /* the TT separable-footprint projector the paper
                               compares with (Sec. I, IV; Long, Fessler &
                               Balter 2010), on the same work split (Sec. V-C):
                               trapezoid footprints across and along the
                               detector columns, integrated over each pixel,
                               times the central ray's chord through the voxel.
                               It estimates the pixel's area-averaged line
                               integral (eq. integ), so it takes
                               CVP_SCALE_COS, elevation_correction 0 and no
                               flags (else CVP_E_INVALID); single-problem entry
                               points only (the batched ones return
                               CVP_E_UNSUPPORTED). */
} cvp_variant;

typedef enum {
    CVP_SCALE_SOLID_ANGLE = 0,  /* unit-sphere formula, eq. cvpus (default) */
    CVP_SCALE_COS = 1,          /* flat-panel formula, eq. cvp */
    CVP_SCALE_NONE = 2          /* unscaled sums S (eq. cvpsu), for tests */
} cvp_scaling;

/* Test mode: weight = cut volume |V^(ijk)_(uv)| (no 1/r^2). */
#define CVP_FLAG_RAW_VOLUME 1u

/* Circular cone-beam geometry.  All lengths in mm, angles in radians. */
typedef struct {
    int32_t vol_dims[3];        /* n1, n2, n3 (> 0) */
    double voxel_mm[3];         /* a1, a2, a3 (> 0) */
    double vol_offset_mm[3];    /* centre of the volume box; 0 = isocentric */
    int32_t det_cols, det_rows; /* M (along chi1), N (along chi2), > 0 */
    double pitch_mm[2];         /* b1, b2 (> 0) */
    double principal_px[2];     /* principal point (pixel-index units);
                                   NAN => ((M-1)/2, (N-1)/2) */
    double source_iso_mm;       /* source-isocentre distance D */
    double source_det_mm;       /* source-detector distance f > D */
    int32_t n_views;            /* >= 1 */
    const double *angles_rad;   /* host pointer, n_views angles; copied */
} cvp_geometry_desc;

typedef struct {
    cvp_variant variant;
    int32_t elevation_correction;   /* 0 off, 1 on (Sec. III-B) */
    cvp_scaling scaling;
    uint32_t flags;                 /* CVP_FLAG_* */
} cvp_options;

typedef struct cvp_geometry cvp_geometry;  /* opaque */

/*
 * Validate a geometry description and build the per-view tables (FP64 on the
 * host, uploaded once to the current HIP device) and the pixel factor tables.
 * Validation: dims > 0, sizes > 0, f > D > half diagonal of the volume box
 * in the x1x2 plane (the source stays outside the volume), n_views >= 1,
 * non-null pointers.  On success *out owns host and device memory; release it
 * with cvp_geometry_destroy.  Errors: CVP_E_INVALID (field named),
 * CVP_E_UNSUPPORTED (projected voxel or volume too large for the kernels),
 * CVP_E_NOMEM, CVP_E_DEVICE.
 */
cvp_status cvp_geometry_from_views(const cvp_geometry_desc *desc, cvp_geometry **out);

/*
 * General trajectory (Sec. III-C: the projective geometry of each view is a
 * camera matrix): one 3x4 matrix per view, row-major, mapping world points
 * (mm, volume as in cvp_geometry_desc) to homogeneous detector coordinates in
 * pixel-index units: (w chi1, w chi2, w) = P (x1, x2, x3, 1); any nonzero
 * scale and either sign.  Supported are the views of the paper's convention
 * (Sec. III-A): chi1 does not depend on x3 (principal ray and chi1 axis
 * horizontal, no skew) and chi2 runs opposite to x3 -- i.e.
 * P = K [R | -R s] with R's rows e1, (0,0,-1), d (e1, d horizontal) and
 * K = [[f/b1, 0, c1], [0, f/b2, c2], [0, 0, 1]]; each view may have its own
 * source position (any height), direction, distances, principal point and
 * pixel aspect (C-arm orbits with wobble).  Views outside the convention
 * give CVP_E_UNSUPPORTED (the message names the view); the volume must lie in
 * front of every source by more than a voxel diagonal (else CVP_E_INVALID).
 * Pixel factors are tabulated per view when views differ in their
 * intrinsics.  Every operator, solver and batch accepts the result like a
 * circular geometry.
 */
typedef struct {
    int32_t vol_dims[3];        /* n1, n2, n3 */
    double voxel_mm[3];
    double vol_offset_mm[3];    /* centre of the volume box */
    int32_t det_cols, det_rows;
    int32_t n_views;
    const double *matrices;     /* host, n_views x 12 doubles (row-major 3x4 per view); copied */
} cvp_geometry_matrices_desc;
cvp_status cvp_geometry_from_matrices(const cvp_geometry_matrices_desc *desc, cvp_geometry **out);

/* Frees the geometry (NULL is ignored).  Not stream-ordered: the caller makes
 * sure no operator call using it is still running. */
void cvp_geometry_destroy(cvp_geometry *g);

/*
 * b = A x.  d_vol: [n3][n2][n1] float32 input; d_proj: [n_views][rows][cols]
 * float32 output, overwritten.  Projection is voxel driven; each workgroup
 * owns a band of detector columns of one view and sums into LDS in 64-bit
 * fixed point, with a scale chosen from the largest |mu| in its wedge, so there
 * are no global atomics and the sums do not depend on the order of the
 * additions: results are bitwise reproducible for a given launch plan.  A
 * non-finite input value makes every band that reads it NaN.
 * Errors: CVP_E_INVALID (null pointer or option), CVP_E_DEVICE (launch).
 */
cvp_status cvp_project(const cvp_geometry *g, const cvp_options *opts,
                       const float *d_vol, float *d_proj, void *hip_stream);

/*
 * cvp_project with caller-provided device scratch: a first kernel stores the
 * largest |mu| of every 16-column group of voxel columns in d_work, and the
 * projection's workgroups take their scales from it instead of reading their
 * volume wedges a second time.  Results equal cvp_project's bitwise.  d_work:
 * work_bytes >= cvp_project_workspace_size bytes (else CVP_E_INVALID),
 * 4-byte aligned, owned by the caller; calls that overlap in time need
 * distinct work buffers.
 */
cvp_status cvp_project_workspace_size(const cvp_geometry *g, int64_t *bytes);
cvp_status cvp_project_ws(const cvp_geometry *g, const cvp_options *opts,
                          const float *d_vol, float *d_proj, void *d_work, int64_t work_bytes,
                          void *hip_stream);

/*
 * cvp_project_ws for callers that cannot allocate (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the per-group
 * maxima live in a fixed device array of the library, CVP_NOALLOC_MAX_GROUPS
 * 32-bit words (1 MiB) per GPU, held until the process ends.  The geometry
 * needs n2 * ceil(n1 / 16) <= CVP_NOALLOC_MAX_GROUPS (else CVP_E_UNSUPPORTED,
 * nothing enqueued).  The call allocates nothing; the first call on a device
 * looks up the array's address there.  Results equal cvp_project_ws's (and
 * cvp_project's) bitwise.  All calls on one GPU share the array: calls that
 * overlap in time on one device (different streams, threads) race and may
 * give wrong results; serialise them, or use cvp_project_ws with distinct
 * work buffers.
 */
#define CVP_NOALLOC_MAX_GROUPS 262144
cvp_status cvp_project_noalloc(const cvp_geometry *g, const cvp_options *opts,
                               const float *d_vol, float *d_proj, void *hip_stream);

/*
 * Reference ray-driven projector SiddonK (Sec. II-D): every pixel of every
 * view gets the mean, over K x K rays from the source to the centres of a
 * K x K grid of equal cells on the pixel, of the line integral of the volume,
 * each line integral the sum of mu times the exact chord length through each
 * voxel the ray crosses (Siddon's parametric traversal), in FP64.  As K grows
 * this tends to the area average of the line integrals over the pixel
 * (eq. integ), which the cutting voxel projector with CVP_SCALE_COS
 * estimates; the paper uses K = 512 as ground truth (Sec. IV-B).  Same
 * geometry, layouts and ownership as cvp_project; output overwritten.  Cost
 * grows as K^2 (rays of pixels outside the projected bounding box of the
 * volume are not traced).  Errors: CVP_E_INVALID (K outside 1..1024, NULL
 * pointer), CVP_E_DEVICE.
 */
cvp_status cvp_project_siddon(const cvp_geometry *g, int32_t K, const float *d_vol, float *d_proj,
                              void *hip_stream);

/*
 * x = A^T b with the same weights (the exact adjoint of cvp_project).
 * d_proj: [n_views][rows][cols] input; d_vol: [n3][n2][n1] output,
 * overwritten.  Voxel-driven gather: every voxel is written once.
 */
cvp_status cvp_backproject(const cvp_geometry *g, const cvp_options *opts,
                           const float *d_proj, float *d_vol, void *hip_stream);

/*
 * The operators restricted to a subset of the geometry's views: views
 * view0, view0 + view_stride, ..., view0 + (n_views - 1) view_stride (all
 * inside 0..n_views of the geometry - 1, else CVP_E_INVALID).  d_proj is the
 * full [n_views][rows][cols] projection array of the geometry: the
 * projection writes only the blocks of the chosen views (the others are left
 * as they are), the backprojection reads only those blocks and returns their
 * adjoint sum.  Ordered subsets of the views (OS-SART, Sec. V-E) use them.
 * cvp_project_views takes optional scratch as cvp_project_ws (d_work NULL:
 * none).  Results equal those of the full operators on the chosen views
 * bitwise.
 */
cvp_status cvp_project_views(const cvp_geometry *g, const cvp_options *opts, const float *d_vol,
                             float *d_proj, int32_t view0, int32_t view_stride, int32_t n_views,
                             void *d_work, int64_t work_bytes, void *hip_stream);
cvp_status cvp_backproject_views(const cvp_geometry *g, const cvp_options *opts, const float *d_proj,
                                 float *d_vol, int32_t view0, int32_t view_stride, int32_t n_views,
                                 void *hip_stream);

/*
 * Batches: several independent problems (each with its own geometry) in one
 * persistent launch per direction.  A fixed grid of workgroups (as many as
 * fit on the GPU) takes work items from an atomic counter until all problems
 * are done, largest items first; every problem's result equals its
 * single-problem result bitwise (each item is summed by one workgroup, in
 * fixed point for the projection and in a fixed order for the
 * backprojection).  The per-call pointer setup and the counter reset are one
 * tiny kernel on the same stream, so a batched call can be graph-captured.
 * n: 1..32 geometries on the same device; the batch keeps pointers to them
 * (they must outlive it) and owns small device tables.  When every member
 * has cached records (cvp_geometry_cache_records) at cvp_batch_create, the
 * batched kernels read them; a call after a member's table was freed or
 * rebuilt returns CVP_E_INVALID.
 */
typedef struct cvp_batch cvp_batch;   /* opaque */
cvp_status cvp_batch_create(const cvp_geometry *const *geoms, int32_t n, cvp_batch **out);
void cvp_batch_destroy(cvp_batch *b);
/* d_vols / d_projs: host arrays of n device pointers (layouts as above).
 * Calls that overlap in time must not share a batch object (it holds the
 * work counter). */
cvp_status cvp_project_batched(const cvp_batch *b, const cvp_options *opts,
                               const float *const *d_vols, float *const *d_projs,
                               void *hip_stream);
cvp_status cvp_backproject_batched(const cvp_batch *b, const cvp_options *opts,
                                   const float *const *d_projs, float *const *d_vols,
                                   void *hip_stream);

/*
 * CGLS on the normal equations A^T A x = A^T b (Hestenes-Stiefel form; the
 * paper times its operators inside CGLS, Sec. IV-A):
 *   start:   r = b - A x,  s = A^T r,  p = s,  gamma = |s|^2
 *   iterate: q = A p,  alpha = gamma/|q|^2,  x += alpha p,  r -= alpha q,
 *            s = A^T r,  gamma' = |s|^2,  p = s + (gamma'/gamma) p
 * Vectors are caller-owned device float32 buffers: x, s, p of volume size;
 * b, r, q of projection size.  The scalars stay on the device, in the
 * caller-owned workspace d_work (cvp_cgls_workspace_size bytes, 8-byte
 * aligned, zeroed once before first use), laid out as doubles:
 *   [0] gamma  [1] |q|^2  [2] alpha  [3] beta  [4] gamma0 = |A^T(b - A x0)|^2
 *   [5] |r|^2  [6] k (iterations done)  [7] breakdown flag (A p = 0 met)
 *   [8] stop flag  [9] gamma threshold of the stop
 *   [10] rho_tol^2 and [11] reference gamma (0: gamma0), set by
 *        cvp_cgls_set_tolerance (0 = never stop)  [12..15] reserved
 *   [16 .. 16+4095]      |s_k|^2 for k = 0..4095
 *   [4112 .. 4112+4095]  |r_k|^2 after iteration k+1
 *   then reduction partials.
 * The relative residual rho_k = sqrt(|s_k|^2 / gamma0) is read from the
 * history.  Stopping on the device: with a tolerance set, cvp_cgls_start
 * fixes the threshold rho_tol^2 * (reference gamma or gamma0) and every
 * iteration raises the stop flag when |s_k|^2 falls to it (or at a
 * breakdown); from then on every kernel of cvp_cgls_iterate returns at once,
 * so x, r and s keep the iterate that met the tolerance through the rest of
 * a captured graph, and k counts the iterations actually run.  Calls enqueue
 * kernels only (no allocation, no host sync), so a run of cvp_cgls_iterate
 * can be captured in a HIP graph.  Dot products accumulate FP64 in a fixed
 * order (bitwise reproducible).
 */
#define CVP_CGLS_HISTORY 4096
cvp_status cvp_cgls_workspace_size(int64_t n_voxels, int64_t n_pixels_total, int64_t *bytes);
/* rho_tol >= 0 (0: never stop), gamma_ref >= 0 (0: the run's own gamma0);
 * takes effect at the next cvp_cgls_start (a one-thread kernel on the stream). */
cvp_status cvp_cgls_set_tolerance(void *d_work, double rho_tol, double gamma_ref, void *hip_stream);
cvp_status cvp_cgls_start(const cvp_geometry *g, const cvp_options *opts, const float *d_b,
                          float *d_x, float *d_r, float *d_s, float *d_p, float *d_q,
                          void *d_work, void *hip_stream);
cvp_status cvp_cgls_iterate(const cvp_geometry *g, const cvp_options *opts, int32_t n_iter,
                            float *d_x, float *d_r, float *d_s, float *d_p, float *d_q,
                            void *d_work, void *hip_stream);

/*
 * Batched CGLS: every problem q of the batch runs the recurrences of
 * cvp_cgls_start / cvp_cgls_iterate on its own vectors and workspace, and
 * each operator step is one batched launch for all problems (the persistent
 * kernels above).  Each problem's iterates and scalars equal those of its
 * single-problem CGLS bitwise.  Arguments are host arrays of b->n device
 * pointers with the single-problem layouts (d_work[q]: cvp_cgls_workspace_size
 * bytes, 8-byte aligned); no vector or workspace may serve two problems.
 * Problems are iterated together; a problem whose stop flag is up (see
 * cvp_cgls_set_tolerance) skips its work items and vector kernels, so the
 * others run on alone.  Enqueues kernels only, so a run of
 * cvp_cgls_batched_iterate can be captured in a HIP graph; calls that overlap
 * in time must not share the batch object.
 */
cvp_status cvp_cgls_batched_start(const cvp_batch *b, const cvp_options *opts, const float *const *d_b,
                                  float *const *d_x, float *const *d_r, float *const *d_s,
                                  float *const *d_p, float *const *d_q, void *const *d_work,
                                  void *hip_stream);
cvp_status cvp_cgls_batched_iterate(const cvp_batch *b, const cvp_options *opts, int32_t n_iter,
                                    float *const *d_x, float *const *d_r, float *const *d_s,
                                    float *const *d_p, float *const *d_q, void *const *d_work,
                                    void *hip_stream);

/*
 * OS-SART (the simultaneous algebraic reconstruction technique of Andersen &
 * Kak over ordered subsets, Jiang & Wang; Sec. V-E of the paper offers it
 * with a subset count) on the same operators.  The views are split into T
 * interleaved subsets S_t = {t, t + T, t + 2T, ...}.  cvp_sart_setup computes
 * the row sums R = A 1 into d_rowsum ([n_views][rows][cols]) and the column
 * sums of every subset C_t = A_t^T 1 into d_colsum (T volumes, one after
 * another), using d_q (projection sized) as scratch.  cvp_sart_iterate runs
 * n_sweeps sweeps over t = 0 .. T-1 of
 *     x <- x + lambda A_t^T ((b_t - A_t x) / R_t) / C_t
 * (a zero denominator gives 0: pixels no voxel reaches, voxels no ray of the
 * subset reaches), then x <- max(x, 0) if nonneg; d_q (projections) and d_z
 * (volume) are scratch.  Caller-owned float32 device buffers, no allocation,
 * no host synchronisation: a run of sweeps can be captured in a HIP graph.
 * Errors: CVP_E_INVALID (T outside 1..n_views, lambda not finite and > 0,
 * aliasing, NULL).
 */
cvp_status cvp_sart_setup(const cvp_geometry *g, const cvp_options *opts, int32_t n_subsets,
                          float *d_rowsum, float *d_colsum, float *d_q, void *hip_stream);
cvp_status cvp_sart_iterate(const cvp_geometry *g, const cvp_options *opts, int32_t n_subsets,
                            int32_t n_sweeps, float lambda, int32_t nonneg, const float *d_b, float *d_x,
                            const float *d_rowsum, const float *d_colsum, float *d_q, float *d_z,
                            void *hip_stream);

/*
 * LSQR (Paige & Saunders, ACM TOMS 8, 1982; Sec. V-E names it next to CGLS):
 * Golub-Kahan bidiagonalisation with a QR update, minimising |b - A x| over
 * growing Krylov spaces (in exact arithmetic the iterates of CGLS).
 *   start:   beta u = b - A x,  alpha v = A^T u,  w = v,
 *            phibar = beta,  rhobar = alpha
 *   iterate: beta u = A v - alpha u,  alpha v = A^T u - beta v,
 *            rho = |(rhobar, beta)|, c = rhobar/rho, s = beta/rho,
 *            x += (c phibar / rho) w,  w = v - (s alpha / rho) w,
 *            rhobar = -c alpha,  phibar = s phibar
 * Vectors: x, v, w, s (volume; s is scratch), u, q (projections; q is
 * scratch).  Scalars on the device in d_work (cvp_lsqr_workspace_size bytes,
 * 8-byte aligned), as doubles: [0] alpha [1] beta [2] rhobar [3] phibar
 * [4] phi/rho [5] theta/rho [6] k (iterations done) [7] end flag (the
 * bidiagonalisation ended; x stays) [8] |A^T (b - A x0)|; from [16]: 4096
 * estimates of |b - A x_k|, then 4096 of |A^T (b - A x_k)| (k = 0, 1, ...),
 * then reduction partials.  No allocation, no host sync: a run of
 * cvp_lsqr_iterate can be captured in a HIP graph.
 */
cvp_status cvp_lsqr_workspace_size(int64_t n_voxels, int64_t n_pixels_total, int64_t *bytes);
cvp_status cvp_lsqr_start(const cvp_geometry *g, const cvp_options *opts, const float *d_b, float *d_x,
                          float *d_u, float *d_v, float *d_w, float *d_q, float *d_s, void *d_work,
                          void *hip_stream);
cvp_status cvp_lsqr_iterate(const cvp_geometry *g, const cvp_options *opts, int32_t n_iter, float *d_x,
                            float *d_u, float *d_v, float *d_w, float *d_q, float *d_s, void *d_work,
                            void *hip_stream);

/* *d_result = sum_i a[i] b[i] accumulated in FP64 (device scalar), using the
 * partials area of a CGLS workspace d_work.  n >= 0. */
cvp_status cvp_dot(const float *d_a, const float *d_b, int64_t n, double *d_result,
                   void *d_work, void *hip_stream);

/*
 * Learned warm start: kernels of a small 3D U-Net (3x3x3 convolutions, BF16
 * activations and weights, FP32 accumulation on the MFMA unit).  Tensors are
 * channels-last BF16 [d][h][w][stride] (channel slices allowed: data points
 * at the first channel, stride = channels of the full tensor); channels and
 * stride are multiples of 8, data 16-byte aligned.  All calls are
 * asynchronous on the stream, allocate nothing, and return CVP_E_INVALID for
 * bad descriptors, CVP_E_UNSUPPORTED for channel counts without a kernel.
 */
typedef struct {
    void *data;
    int32_t d, h, w;
    int32_t channels;
    int32_t stride;
} cvp_nn_tensor;

/* out = [relu](conv3d(in, W) + bias), 3x3x3, zero padding 1.  weight: BF16
 * [27][Cout][Cin] (tap = 9 dz + 3 dy + dx); Cout in {16, 32, 64}.  flip = 1
 * mirrors the taps: with weights from cvp_nn_transpose_weights this is the
 * backward-data convolution. */
cvp_status cvp_nn_conv3d(const cvp_nn_tensor *in, const void *weight, const float *bias,
                         const cvp_nn_tensor *out, int32_t relu, int32_t flip, void *stream);
/* dW[tap][co][ci] = sum_v dY[v][co] X[v + off(tap)][ci] (FP32), via per-chunk
 * partials in work (cvp_nn_wgrad_workspace floats) and a fixed-order sum. */
cvp_status cvp_nn_wgrad_workspace(const cvp_nn_tensor *x, const cvp_nn_tensor *dy, int64_t *floats);
cvp_status cvp_nn_conv3d_wgrad(const cvp_nn_tensor *x, const cvp_nn_tensor *dy, float *dw, float *work,
                               int64_t work_floats, void *stream);
/* out[c] = sum_v a[v][c] (bias gradient); work >= ceil(d*h/16) * channels floats */
cvp_status cvp_nn_channel_sum(const cvp_nn_tensor *a, float *out, float *work, int64_t work_floats,
                              void *stream);
/* dy[v][c] = 0 where y[v][c] <= 0 (ReLU backward from the post-ReLU output) */
cvp_status cvp_nn_relu_mask(const cvp_nn_tensor *dy, const cvp_nn_tensor *y, void *stream);
cvp_status cvp_nn_avgpool2(const cvp_nn_tensor *in, const cvp_nn_tensor *out, void *stream);
cvp_status cvp_nn_avgpool2_bwd(const cvp_nn_tensor *dout, const cvp_nn_tensor *din, void *stream);
cvp_status cvp_nn_upsample2(const cvp_nn_tensor *in, const cvp_nn_tensor *out, void *stream);
cvp_status cvp_nn_upsample2_bwd(const cvp_nn_tensor *dout, const cvp_nn_tensor *din, void *stream);
/* out = a + b (BF16, same shape) */
cvp_status cvp_nn_add(const cvp_nn_tensor *a, const cvp_nn_tensor *b, const cvp_nn_tensor *out,
                      void *stream);
/* wt[tap][ci][co] = w[tap][co][ci] (BF16) */
cvp_status cvp_nn_transpose_weights(const void *w, void *wt, int32_t cout, int32_t cin, void *stream);
/* out channels 0, 1 = scale * x1, scale * x2 (FP32 volumes); channels 2..15 = 0 */
cvp_status cvp_nn_pack_input(const float *x1, const float *x2, float scale, const cvp_nn_tensor *out,
                             void *stream);
/* x0 = x2 + (sum_c w[c] h[v][c] + b[0]) / scale  (1x1x1 head, residual on x2) */
cvp_status cvp_nn_head(const cvp_nn_tensor *h, const float *w, const float *b, const float *x2,
                       float scale, float *x0, void *stream);
/* head backward: dh = w g / scale (BF16); dwb[0..15] = dL/dw, dwb[16] = dL/db */
cvp_status cvp_nn_head_bwd(const cvp_nn_tensor *h, const float *w, const float *g, float scale,
                           const cvp_nn_tensor *dh, float *dwb, float *work, int64_t work_floats,
                           void *stream);
/* grad = 2 (a - b) / n, *loss = mean (a - b)^2 (device FP64); work >= 1024 doubles */
cvp_status cvp_nn_mse(const float *a, const float *b, int64_t n, float *grad, double *loss,
                      double *work, int64_t work_doubles, void *stream);
/* Adam step on FP32 parameters (bias-corrected, step >= 1), optional BF16 copy */
cvp_status cvp_nn_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr,
                       float beta1, float beta2, float eps, int32_t step, void *p_bf16,
                       void *stream);

/*
 * Synthetic inputs on the device (training data of the warm start; not part
 * of the operator).  cvp_synth_ellipsoids: vol[k][j][i] = sum of mu over the
 * ellipsoids containing the voxel centre ((i - (n1-1)/2) a1, ...); d_params is
 * a device array of n x 16 doubles (centre, semi-axes, row-major rotation
 * body -> world, mu), evaluated in FP64 without contraction.
 * cvp_synth_add_gaussian: out[i] += sigma * N(0,1), Philox4x32-10 with
 * counter i/4 and key seed, Box-Muller.
 */
cvp_status cvp_synth_ellipsoids(const double *d_params, int32_t n, const int32_t dims[3],
                                const double voxel_mm[3], float *d_vol, void *hip_stream);
cvp_status cvp_synth_add_gaussian(float *d_out, int64_t n, float sigma, uint64_t seed,
                                  void *hip_stream);

/* Launch plan of a geometry: how the work is split, never what is computed.
 *   proj_band_cols  detector columns per projection work item (1..32); the
 *                   work item's fixed-point band image takes 8 bytes per
 *                   detector row and column of LDS (at most 156 KB in all), so
 *                   small values let more workgroups share a compute unit.
 *   bp_stack_cols   voxel columns per backprojection workgroup (16, 8 or 4).
 *   bp_passes       64-voxel passes per backprojection stack (1 or 2): two
 *                   passes share each view's piece records and detector
 *                   window, one keeps the window small enough for LDS.
 *   bp_workgroups_per_cu  with cached records (cvp_geometry_cache_records):
 *                   backprojection workgroups the LDS budget is sized for, 4
 *                   (40 KB each) or 3 (52 KB each, larger detector windows);
 *                   the default is 4 for 4-piece records, 3 for 8-piece ones.
 *                   Records computed in the kernel always take 52 KB (3); it
 *                   is reported as such.
 *   bp_shared_window  with cached records and stacks of 8 or 16 columns: 1
 *                   stages one detector window per workgroup (all four waves
 *                   on one view at a time, each window four times as large
 *                   as a wave's own: for detectors whose pixels are small
 *                   against the voxels), 0 (the default) one per wave.  A
 *                   request the plan cannot honour (no cached records,
 *                   4-column stacks) is reported as 0.
 * cvp_geometry_get_launch reports the plan in use (the planner's default
 * after cvp_geometry_from_views).  cvp_geometry_set_launch replaces it; a zero
 * field restores the default for that field.  Errors: CVP_E_INVALID (NULL or a
 * value outside the sets above), CVP_E_UNSUPPORTED (the plan does not fit
 * LDS); the plan is unchanged on error.  Set the plan while no other call
 * uses the geometry; launches already enqueued keep the plan they were
 * given, and batches keep the plans of their members at cvp_batch_create.
 * Results of a given plan are bitwise reproducible; backprojections do not
 * depend on the plan at all, while two plans may differ in the last bit of a
 * few projection values (the fixed-point scale of a work item depends on the
 * part of the volume it reads). */
typedef struct {
    int32_t proj_band_cols;
    int32_t bp_stack_cols;
    int32_t bp_passes;
    int32_t bp_workgroups_per_cu;
    int32_t bp_shared_window;
} cvp_launch;

cvp_status cvp_geometry_get_launch(const cvp_geometry *g, cvp_launch *out);
cvp_status cvp_geometry_set_launch(cvp_geometry *g, const cvp_launch *in);

/* Geometry queries (host-side, no device work). */
cvp_status cvp_geometry_sizes(const cvp_geometry *g, int64_t *n_voxels,
                              int64_t *n_pixels_total);

/* Cache the geometry's cut-piece records (Sec. III-A: by the column identity
 * a voxel column's polygons H_u in one view serve every voxel of the column).
 * enable = 1 computes, once, for every view and every voxel column (i, j)
 * the FP64 polygon moments of its pieces (detector columns in [0, M - 1]) and
 * keeps the resulting records on the geometry's device: n_views * n2 * n1 *
 * (pmax * 48 + 4) bytes, pmax = 4 or 8 pieces per column (12.7 GB for 512^3
 * voxels and 248 views).  From then on cvp_project, cvp_backproject, their
 * _ws / _views / _noalloc variants and the solvers of the cutting voxel
 * projector (both forms, EC on or off) read the records instead of computing
 * them in each launch; results are bitwise the same.  The TT projector and
 * the batched launches keep computing their own.  Without its FP64 stage the
 * backprojection needs less LDS per workgroup, so its plan is re-derived for a
 * smaller LDS budget (the same stack shape when it fits; likewise back when
 * the table is freed).  enable = 0 frees the table.
 * *bytes (may be NULL) receives the table's size.  The fill is enqueued on
 * `stream`; it allocates (hipMalloc) on the first enable only.  Call it while
 * no other call uses the geometry.  Errors: CVP_E_INVALID (NULL geometry,
 * enable not 0 or 1, another device current), CVP_E_UNSUPPORTED (voxels
 * projecting onto more than 8 detector columns), CVP_E_NOMEM, CVP_E_DEVICE. */
cvp_status cvp_geometry_cache_records(cvp_geometry *g, int32_t enable, int64_t *bytes, void *stream);

/* Human-readable status name; never NULL. */
const char *cvp_status_string(cvp_status s);

/* Copies the calling thread's last error message into buf (NUL-terminated,
 * truncated to n bytes).  Returns CVP_OK, or CVP_E_INVALID if buf is NULL. */
cvp_status cvp_last_error_detail(char *buf, size_t n);

#ifdef __cplusplus
}
#endif

#endif /* CVP_H */
