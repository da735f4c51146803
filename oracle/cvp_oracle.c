/*
 * Cutting voxel projector (CVP) -- plain FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load or call this file.  The product path
 * (the HIP library) neither links nor includes it, and it shares no code,
 * header, table or constant generator with that path.
 *
 * What it computes (Kulvait & Rose, "Cutting Voxel Projector a New Approach to
 * Construct 3D Cone Beam CT Operator", 2021):
 *
 *   b = A x,   x = A^T b,
 *   A[(view,v,u),(i,j,k)] = sigma_uv * |V^(ijk)_(uv)| / r^2
 *
 * where |V^(ijk)_(uv)| is the paper's estimate of the volume of the voxel cut
 * by the ray pyramid of pixel (u,v) (Sec. III-A, eq. cutvolume, optionally with
 * the elevation correction of Sec. III-B), 1/r^2 is the approximation of the
 * cut integral of 1/r^2 (Sec. II-F, eq. vox), and sigma_uv is the per-pixel
 * factor of the flat-panel formula (Sec. II-E, eq. cvp) or of the unit-sphere
 * formula (eq. cvpus), applied after the unscaled sums (eq. cvpsu).
 *
 * CVP is an approximation, so this oracle follows the paper's steps in the
 * paper's order, in FP64, with no blocking, fusion or reordering:
 *   1. per view, the source-centred frame Q (Sec. II-C);
 *   2. per voxel column (i,j), the polygons H_u of the voxel base cut by the
 *      column strips u-1/2 <= chi1 <= u+1/2 (Sec. III-A; the column identity
 *      eq. columnprojectionidentity makes them the same for every k);
 *      this oracle clips each strip directly, the area A_u and centroid CM_u
 *      come from the polygon formulas;
 *   3. per voxel, the x3 extent of the cut at the centroid depth for every
 *      detector row (Sec. III-A), or its average over a depth box (Sec. III-B);
 *   4. weight vol/r^2 (Sec. II-F), summed into S (eq. cvpsu);
 *   5. pixel scaling (Sec. III-C, "second phase").
 *
 * Readings of points the paper leaves open (all listed with reasons in the
 * design notes of the repository):
 *   - pixel (u,v): u along chi1 (column), v along chi2 (row), in pixel-index
 *     units, pixel (u,v) covers [u-1/2,u+1/2] x [v-1/2,v+1/2];
 *   - circular orbit about +x3: s = (D cos l, D sin l, 0), rows of Q are
 *     e1 = (-sin l, cos l, 0), e2 = (0,0,-1) (chi2 opposite to x3, Sec. III-A),
 *     d = (-cos l, -sin l, 0);
 *   - exact form: r at the centroid of the cut piece; relaxed form: r at the
 *     voxel centre (the two choices of r named in Sec. II-F);
 *   - elevation correction: the cut is represented by a rectangle in the
 *     plane chi1 = const, symmetric about the centroid (Sec. III-B); its half
 *     width in depth is h = sqrt(3 Var_H(D)), the half width of the uniform
 *     box with the same depth variance as the polygon H_u.  PARITY UNPINNED
 *     against the paper's own implementation (the paper calls its width a
 *     heuristic and does not give it); only invariants pin it.
 *   - pixels off the detector are dropped (no renormalisation).
 *
 * General trajectories (Sec. III-C: per-view camera matrices, under the
 * convention of Sec. III-A that chi2 runs opposite to x3): instead of the
 * circular orbit, each view may come with its own frame and intrinsics
 * (source s, horizontal e1 and d, e2 = (0,0,-1), f/b1, f/b2, principal
 * point), taken from its projection matrix by the Python side.  Every
 * formula above is unchanged; only the constants become per view.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t n1, n2, n3;     /* voxels per edge, x1 fastest in memory */
    double a1, a2, a3;      /* voxel size [mm] */
    double o1, o2, o3;      /* centre of the volume box [mm] */
    int32_t ncols, nrows;   /* M pixels along chi1, N pixels along chi2 */
    double b1, b2;          /* pixel pitch [mm] */
    double c1, c2;          /* principal point, pixel-index units */
    double sid, sdd;        /* source-isocentre, source-detector [mm] */
    int32_t nviews;
    const double *angles;   /* [nviews] rotation angles [rad] */
    const double *frames;   /* NULL (circular orbit) or [nviews][11]: s1, s2, s3,
                               e1x, e1y, dx, dy, f/b1, f/b2, c1, c2 */
} orc_geom;

typedef struct {
    int32_t exact;          /* 1: r at the cut centroid; 0: at the voxel centre */
    int32_t ec;             /* elevation correction on/off */
    int32_t scaling;        /* 0: unit sphere (eq. cvpus), 1: flat panel (eq. cvp), 2: none */
    int32_t raw_volume;     /* 1: weight = cut volume (no 1/r^2) */
} orc_opts;

typedef struct {
    int32_t u;              /* detector column */
    double area;            /* A_u */
    double cm1, cm2;        /* centroid CM_u (world x1, x2) */
    double depth;           /* D_u = d . (CM_u - s) */
    double h;               /* elevation-correction half width (0 if off) */
} orc_piece;

/* Deliberate mistakes, switched on only by the mutation tests to show that
 * the pins catch them.  0 = none. */
static int g_mutation = 0;
void orc_set_mutation(int m) { g_mutation = m; }

/* ---------------------------------------------------------------- frames */

/* Sec. II-C: x~ = Q (x - s); rows of Q are e1 (parallel to chi1), e2
 * (parallel to chi2) and d (principal ray, source to detector). */
static void view_frame(const orc_geom *g, int view, double s[3], double e1[3],
                       double e2[3], double d[3])
{
    if (g->frames) {
        const double *F = g->frames + (size_t)view * 11;
        s[0] = F[0]; s[1] = F[1]; s[2] = F[2];
        e1[0] = F[3]; e1[1] = F[4]; e1[2] = 0.0;
        e2[0] = 0.0; e2[1] = 0.0; e2[2] = -1.0;
        d[0] = F[5]; d[1] = F[6]; d[2] = 0.0;
        if (g_mutation == 1) { e1[0] = -e1[0]; e1[1] = -e1[1]; }
        return;
    }
    double l = g->angles[view];
    double cl = cos(l), sl = sin(l);
    s[0] = g->sid * cl; s[1] = g->sid * sl; s[2] = 0.0;
    e1[0] = -sl; e1[1] = cl;  e1[2] = 0.0;
    e2[0] = 0.0; e2[1] = 0.0; e2[2] = -1.0;
    d[0] = -cl;  d[1] = -sl;  d[2] = 0.0;
    if (g_mutation == 1) { e1[0] = sl; e1[1] = -cl; }   /* mirrored detector */
}

void orc_view_frame(const orc_geom *g, int view, double *s, double *e1,
                    double *e2, double *d)
{
    view_frame(g, view, s, e1, e2, d);
}

static double dot3(const double *a, const double *b)
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* Intrinsics of a view in pixel-index units: fb1 = f/b1, fb2 = f/b2 (and its
 * inverse b2/f), principal point (c1, c2). */
typedef struct {
    double fb1, fb2, ifb2, c1, c2;
} orc_intr;

static orc_intr view_intr(const orc_geom *g, int view)
{
    orc_intr I;
    if (g->frames) {
        const double *F = g->frames + (size_t)view * 11;
        I.fb1 = F[7]; I.fb2 = F[8]; I.ifb2 = 1.0 / F[8]; I.c1 = F[9]; I.c2 = F[10];
    } else {
        I.fb1 = g->sdd / g->b1; I.fb2 = g->sdd / g->b2; I.ifb2 = g->b2 / g->sdd;
        I.c1 = g->c1; I.c2 = g->c2;
    }
    return I;
}

/* pinhole projection of a world point onto detector pixel-index coordinates */
void orc_project_point(const orc_geom *g, int view, const double *x, double *chi)
{
    double s[3], e1[3], e2[3], d[3], r[3];
    view_frame(g, view, s, e1, e2, d);
    r[0] = x[0] - s[0]; r[1] = x[1] - s[1]; r[2] = x[2] - s[2];
    double depth = dot3(d, r);
    const orc_intr I = view_intr(g, view);
    chi[0] = I.c1 + I.fb1 * dot3(e1, r) / depth;
    chi[1] = I.c2 + I.fb2 * dot3(e2, r) / depth;
}

static void voxel_centre(const orc_geom *g, int i, int j, int k, double x[3])
{
    /* Sec. II-A: x^(000) = (-l + a)/2, x^(ijk) = x^(000) + (i a1, j a2, k a3),
     * shifted by the volume offset. */
    x[0] = g->o1 + 0.5 * (-g->n1 * g->a1 + g->a1) + i * g->a1;
    x[1] = g->o2 + 0.5 * (-g->n2 * g->a2 + g->a2) + j * g->a2;
    x[2] = g->o3 + 0.5 * (-g->n3 * g->a3 + g->a3) + k * g->a3;
}

/* ------------------------------------------------------- 2D polygon cuts */

#define MAXV 16

/* Sutherland-Hodgman clip of polygon p (n vertices) against the half-plane
 * {q : sgn * (nx*q.x + ny*q.y + c) <= 0}. */
static int clip_halfplane(const double (*p)[2], int n, double nx, double ny,
                          double c, double sgn, double (*out)[2])
{
    int m = 0;
    for (int a = 0; a < n; ++a) {
        int b = (a + 1) % n;
        double fa = sgn * (nx * p[a][0] + ny * p[a][1] + c);
        double fb = sgn * (nx * p[b][0] + ny * p[b][1] + c);
        if (fa <= 0) { out[m][0] = p[a][0]; out[m][1] = p[a][1]; ++m; }
        if ((fa < 0 && fb > 0) || (fa > 0 && fb < 0)) {
            double t = fa / (fa - fb);
            out[m][0] = p[a][0] + t * (p[b][0] - p[a][0]);
            out[m][1] = p[a][1] + t * (p[b][1] - p[a][1]);
            ++m;
        }
    }
    return m;
}

/* area, first and central second moments of a simple polygon (vertices in
 * counter-clockwise order) by the shoelace / Green's theorem formulas */
static void polygon_moments(const double (*p)[2], int n, double *area,
                            double *cx, double *cy, double *sxx, double *sxy,
                            double *syy)
{
    double A = 0, Mx = 0, My = 0, Ixx = 0, Ixy = 0, Iyy = 0;
    for (int a = 0; a < n; ++a) {
        int b = (a + 1) % n;
        double x0 = p[a][0], y0 = p[a][1], x1 = p[b][0], y1 = p[b][1];
        double cr = x0 * y1 - x1 * y0;
        A += cr;
        Mx += (x0 + x1) * cr;
        My += (y0 + y1) * cr;
        Ixx += (x0 * x0 + x0 * x1 + x1 * x1) * cr;
        Iyy += (y0 * y0 + y0 * y1 + y1 * y1) * cr;
        Ixy += (x0 * y1 + 2 * x0 * y0 + 2 * x1 * y1 + x1 * y0) * cr;
    }
    A *= 0.5;
    *area = A;
    if (A <= 0) { *cx = *cy = *sxx = *sxy = *syy = 0; return; }
    *cx = Mx / (6 * A);
    *cy = My / (6 * A);
    /* raw second moments  int x^2 dA = Ixx/12 etc., then centred */
    *sxx = Ixx / 12 - A * (*cx) * (*cx);
    *syy = Iyy / 12 - A * (*cy) * (*cy);
    *sxy = Ixy / 24 - A * (*cx) * (*cy);
}

/*
 * Sec. III-A: the voxel base B of column (i,j) is cut by the rays to the
 * detector columns.  Column u collects the points with u-1/2 <= chi1 <= u+1/2.
 * chi1 <= t  <=>  n_t . (x - s) <= 0  with  n_t = (f/b1) e1 - (t - c1) d,
 * because d.(x-s) > 0 in front of the source.  Returns the pieces H_u with
 * non-zero area, for detector columns inside [0, M).
 */
int orc_column_pieces(const orc_geom *g, const orc_opts *o, int view, int i,
                      int j, orc_piece *out, int max_out)
{
    double s[3], e1[3], e2[3], d[3], xc[3];
    view_frame(g, view, s, e1, e2, d);
    voxel_centre(g, i, j, 0, xc);
    const orc_intr I = view_intr(g, view);

    /* chi1 of the four base corners -> range of detector columns */
    double chimin = INFINITY, chimax = -INFINITY;
    for (int c = 0; c < 4; ++c) {
        double x[3] = {xc[0] + ((c & 1) ? 0.5 : -0.5) * g->a1,
                       xc[1] + ((c & 2) ? 0.5 : -0.5) * g->a2, 0.0};
        double chi[2];
        orc_project_point(g, view, x, chi);
        if (chi[0] < chimin) chimin = chi[0];
        if (chi[0] > chimax) chimax = chi[0];
    }
    int ulo = (int)floor(chimin + 0.5), uhi = (int)floor(chimax + 0.5);
    const int ulo_all = ulo, uhi_all = uhi;
    if (ulo < 0) ulo = 0;
    if (uhi > g->ncols - 1) uhi = g->ncols - 1;

    /* base square in coordinates local to the column centre, CCW */
    double sq[4][2] = {{-0.5 * g->a1, -0.5 * g->a2}, {0.5 * g->a1, -0.5 * g->a2},
                       {0.5 * g->a1, 0.5 * g->a2},   {-0.5 * g->a1, 0.5 * g->a2}};
    double rc[2] = {xc[0] - s[0], xc[1] - s[1]};

    int np = 0;
    for (int u = ulo; u <= uhi; ++u) {
        double tl = u - 0.5, th = u + 0.5;
        if (g_mutation == 2) th = u + 0.6;              /* wrong pixel edge */
        /* n_t in the x1x2 plane; the half-plane test on local q is
         * n_t.q + n_t.(x_c - s) */
        double nl0 = I.fb1 * e1[0] - (tl - I.c1) * d[0];
        double nl1 = I.fb1 * e1[1] - (tl - I.c1) * d[1];
        double nh0 = I.fb1 * e1[0] - (th - I.c1) * d[0];
        double nh1 = I.fb1 * e1[1] - (th - I.c1) * d[1];
        double p1[MAXV][2], p2[MAXV][2];
        /* chi1 >= u - 1/2 : -(n.(x-s)) <= 0 */
        int n1 = clip_halfplane((const double (*)[2])sq, 4, nl0, nl1,
                                nl0 * rc[0] + nl1 * rc[1], -1.0, p1);
        if (g_mutation == 7 && u == ulo && ulo_all < ulo) {
            /* the part left of the detector merged into its first column */
            memcpy(p1, sq, sizeof(sq));
            n1 = 4;
        }
        /* chi1 <= u + 1/2 */
        int n2 = clip_halfplane((const double (*)[2])p1, n1, nh0, nh1,
                                nh0 * rc[0] + nh1 * rc[1], 1.0, p2);
        if (g_mutation == 7 && u == uhi && uhi_all > uhi) {
            memcpy(p2, p1, sizeof(p1));
            n2 = n1;
        }
        if (n2 < 3) continue;
        double A, cx, cy, sxx, sxy, syy;
        polygon_moments((const double (*)[2])p2, n2, &A, &cx, &cy, &sxx, &sxy, &syy);
        if (!(A > 0)) continue;
        if (np >= max_out) return -1;
        orc_piece *pc = &out[np++];
        pc->u = u;
        pc->area = A;
        pc->cm1 = xc[0] + cx;
        pc->cm2 = xc[1] + cy;
        pc->depth = d[0] * (pc->cm1 - s[0]) + d[1] * (pc->cm2 - s[1]);
        if (g_mutation == 3) pc->depth = d[0] * (xc[0] - s[0]) + d[1] * (xc[1] - s[1]);
        if (o->ec) {
            /* variance of the depth D(x) = d.(x-s) over H_u */
            double var = (d[0] * d[0] * sxx + 2 * d[0] * d[1] * sxy + d[1] * d[1] * syy) / A;
            pc->h = var > 0 ? sqrt(3.0 * var) : 0.0;
        } else {
            pc->h = 0.0;
        }
    }
    return np;
}

/* ---------------------------------------------------------- row extents */

/* x3 of the plane through the source onto the row boundary chi2 = t, at
 * depth Dp:  chi2 = c2 + (f/b2) e2.(x-s)/Dp  with e2 = (0,0,-1). */
static double row_plane_x3(const orc_intr *I, double s3, double t, double Dp)
{
    return s3 - (t - I->c2) * I->ifb2 * Dp;
}

/* Sec. III-A: x3 length of [z0,z1] inside the band of row v at depth Dp. */
static double band_length(const orc_intr *I, double s3, int v, double Dp,
                          double z0, double z1)
{
    double top = row_plane_x3(I, s3, v - 0.5, Dp);
    double bot = row_plane_x3(I, s3, v + 0.5, Dp);
    if (g_mutation == 4) bot = row_plane_x3(I, s3, v + 0.5, Dp * 1.001);
    double lo = z0 > bot ? z0 : bot;
    double hi = z1 < top ? z1 : top;
    return hi > lo ? hi - lo : 0.0;
}

static int cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* Sec. III-B: the cut is represented by a rectangle [D-h, D+h] x [z0, z1] in
 * the plane of constant chi1; the row gets the mean of band_length over the
 * depth box.  The integrand is piecewise linear in Dp with kinks only where
 * a row plane passes z0 or z1, so the trapezoid rule between those kinks is
 * exact. */
double orc_row_length(const orc_geom *g, int view, double s3, int v, double D, double h,
                      double z0, double z1)
{
    const orc_intr I = view_intr(g, view);
    if (!(h > 0)) return band_length(&I, s3, v, D, z0, z1);
    double bp[8];
    int nb = 0;
    bp[nb++] = D - h;
    bp[nb++] = D + h;
    const double ts[2] = {v - 0.5, v + 0.5};
    const double zs[2] = {z0, z1};
    for (int a = 0; a < 2; ++a) {
        double k = (ts[a] - I.c2) * I.ifb2;
        if (k == 0) continue;
        for (int b = 0; b < 2; ++b) {
            double Dp = (s3 - zs[b]) / k;
            if (Dp > D - h && Dp < D + h) bp[nb++] = Dp;
        }
    }
    qsort(bp, nb, sizeof(double), cmp_double);
    double acc = 0;
    for (int a = 0; a + 1 < nb; ++a) {
        double w = bp[a + 1] - bp[a];
        if (w <= 0) continue;
        acc += 0.5 * w * (band_length(&I, s3, v, bp[a], z0, z1) +
                          band_length(&I, s3, v, bp[a + 1], z0, z1));
    }
    /* mean over the box; its width as represented (bp[nb-1] - bp[0]) rather
     * than 2h keeps the quotient exact for boxes narrower than the FP64
     * spacing of D */
    return acc / (bp[nb - 1] - bp[0]);
}

/* ------------------------------------------------------- voxel weights */

/*
 * All (u, v, w) of voxel (i,j,k) in a view, where w is the weight of the
 * voxel in the unscaled sum S_uv (eq. cvpsu): A_u d_uv / r^2 (eq. cutvolume
 * and eq. vox), or A_u d_uv with raw_volume.  Returns the count, -1 on
 * overflow.
 */
int orc_voxel_weights(const orc_geom *g, const orc_opts *o, int view, int i,
                      int j, int k, int32_t *us, int32_t *vs, double *ws,
                      int max_out)
{
    orc_piece pcs[64];
    int np = orc_column_pieces(g, o, view, i, j, pcs, 64);
    if (np < 0) return -1;
    double s[3], e1[3], e2[3], d[3], xc[3];
    view_frame(g, view, s, e1, e2, d);
    voxel_centre(g, i, j, k, xc);
    const orc_intr I = view_intr(g, view);
    double z0 = xc[2] - 0.5 * g->a3, z1 = xc[2] + 0.5 * g->a3;
    int n = 0;
    double volsum = 0.0;
    for (int p = 0; p < np; ++p) {
        const orc_piece *pc = &pcs[p];
        double h = pc->h;
        /* rows reached by the box corners (depth D +- h, height z0, z1) */
        double cmin = INFINITY, cmax = -INFINITY;
        for (int a = 0; a < 4; ++a) {
            double Dp = pc->depth + ((a & 1) ? h : -h);
            double z = (a & 2) ? z1 : z0;
            double chi2 = I.c2 - I.fb2 * (z - s[2]) / Dp;
            if (chi2 < cmin) cmin = chi2;
            if (chi2 > cmax) cmax = chi2;
        }
        int vlo = (int)floor(cmin + 0.5), vhi = (int)floor(cmax + 0.5);
        const int vlo_all = vlo, vhi_all = vhi;
        if (vlo < 0) vlo = 0;
        if (vhi > g->nrows - 1) vhi = g->nrows - 1;
        for (int v = vlo; v <= vhi; ++v) {
            double len = orc_row_length(g, view, s[2], v, pc->depth, h, z0, z1);
            if (g_mutation == 9) {
                /* rows off the detector merged into its edge rows */
                if (v == vlo)
                    for (int vv = vlo_all; vv < vlo; ++vv) len += orc_row_length(g, view, s[2], vv, pc->depth, h, z0, z1);
                if (v == vhi)
                    for (int vv = vhi + 1; vv <= vhi_all; ++vv) len += orc_row_length(g, view, s[2], vv, pc->depth, h, z0, z1);
            }
            volsum += pc->area * len;
            if (!(len > 0)) continue;
            double vol = pc->area * len;              /* eq. cutvolume */
            double w;
            if (o->raw_volume) {
                w = vol;
            } else {
                double r2;
                if (o->exact) {
                    /* centroid of the piece: CM_u in x1x2, middle of the x3
                     * extent of the plain band at the centroid depth */
                    double top = row_plane_x3(&I, s[2], v - 0.5, pc->depth);
                    double bot = row_plane_x3(&I, s[2], v + 0.5, pc->depth);
                    double lo = z0 > bot ? z0 : bot, hi = z1 < top ? z1 : top;
                    double zb = 0.5 * (lo + hi);
                    if (zb < z0) zb = z0;
                    if (zb > z1) zb = z1;
                    double q0 = pc->cm1 - s[0], q1 = pc->cm2 - s[1], q2 = zb - s[2];
                    r2 = q0 * q0 + q1 * q1 + q2 * q2;
                } else {
                    double q0 = xc[0] - s[0], q1 = xc[1] - s[1], q2 = xc[2] - s[2];
                    r2 = q0 * q0 + q1 * q1 + q2 * q2;
                }
                w = vol / r2;                          /* eq. vox */
                if (g_mutation == 5) w = vol / sqrt(r2);
            }
            if (n >= max_out) return -1;
            us[n] = pc->u; vs[n] = v; ws[n] = w; ++n;
        }
    }
    if (g_mutation == 8 && volsum > 0) {
        /* renormalised to the whole voxel volume when parts were dropped */
        double fix = g->a1 * g->a2 * g->a3 / volsum;
        for (int q = 0; q < n; ++q) ws[q] *= fix;
    }
    return n;
}

/* ------------------------------------------------------ pixel scaling */

/* Solid angle of the triangle (0, A, B, C) seen from the origin, by the
 * formula of Van Oosterom and Strackee (1983). */
static double tri_solid_angle(const double *A, const double *B, const double *C)
{
    double la = sqrt(dot3(A, A)), lb = sqrt(dot3(B, B)), lc = sqrt(dot3(C, C));
    double bxc[3] = {B[1] * C[2] - B[2] * C[1], B[2] * C[0] - B[0] * C[2],
                     B[0] * C[1] - B[1] * C[0]};
    double num = fabs(dot3(A, bxc));
    double den = la * lb * lc + dot3(A, B) * lc + dot3(A, C) * lb + dot3(B, C) * la;
    return 2.0 * atan2(num, den);
}

/* Solid angle of pixel (u,v) of a view seen from the source: the detector
 * plane is at distance f along the principal ray, pixel edges at (t - c) * b
 * (with per-view frames: at distance 1, edges at (t - c) / (f/b)). */
double orc_pixel_solid_angle_view(const orc_geom *g, int view, int u, int v)
{
    double x0, x1, y0, y1, f;
    if (g->frames) {
        const orc_intr I = view_intr(g, view);
        x0 = (u - 0.5 - I.c1) / I.fb1; x1 = (u + 0.5 - I.c1) / I.fb1;
        y0 = (v - 0.5 - I.c2) / I.fb2; y1 = (v + 0.5 - I.c2) / I.fb2;
        f = 1.0;
    } else {
        x0 = (u - 0.5 - g->c1) * g->b1; x1 = (u + 0.5 - g->c1) * g->b1;
        y0 = (v - 0.5 - g->c2) * g->b2; y1 = (v + 0.5 - g->c2) * g->b2;
        f = g->sdd;
    }
    double P[4][3] = {{x0, y0, f}, {x1, y0, f}, {x1, y1, f}, {x0, y1, f}};
    return tri_solid_angle(P[0], P[1], P[2]) + tri_solid_angle(P[0], P[2], P[3]);
}

double orc_pixel_solid_angle(const orc_geom *g, int u, int v)
{
    return orc_pixel_solid_angle_view(g, 0, u, v);
}

/* Sec. III-C, second phase: the factor applied to S_uv per pixel of a view.
 *   scaling 0: 1 / abar_uv                  (eq. cvpus)
 *   scaling 1: f^2 / (a_uv cos^3 theta_uv)  (eq. cvp), theta at the pixel centre
 *   scaling 2: 1 */
void orc_pixel_scale_view(const orc_geom *g, int view, int scaling, double *sigma)
{
    for (int v = 0; v < g->nrows; ++v) {
        for (int u = 0; u < g->ncols; ++u) {
            double val = 1.0;
            if (scaling == 0) {
                val = 1.0 / orc_pixel_solid_angle_view(g, view, u, v);
            } else if (scaling == 1) {
                if (g->frames) {
                    const orc_intr I = view_intr(g, view);
                    double X = (u - I.c1) / I.fb1, Y = (v - I.c2) / I.fb2;
                    double cth = 1.0 / sqrt(X * X + Y * Y + 1.0);
                    val = I.fb1 * I.fb2 / (cth * cth * cth);
                } else {
                    double X = (u - g->c1) * g->b1, Y = (v - g->c2) * g->b2;
                    double R = sqrt(X * X + Y * Y + g->sdd * g->sdd);
                    double cth = g->sdd / R;
                    val = g->sdd * g->sdd / (g->b1 * g->b2 * cth * cth * cth);
                }
            }
            sigma[(size_t)v * g->ncols + u] = val;
        }
    }
}

void orc_pixel_scale(const orc_geom *g, int scaling, double *sigma)
{
    orc_pixel_scale_view(g, 0, scaling, sigma);
}

/* ---------------------------------------------------------- operators */

static int nthreads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static int thread_id(void)
{
#ifdef _OPENMP
    return omp_get_thread_num();
#else
    return 0;
#endif
}

#define MAXW 4096

/*
 * b = A x for views [view_lo, view_hi).  x: [n3][n2][n1], b: [views][nrows][ncols].
 * Each thread sums into its own detector image; the images are added at the
 * end of each view.
 */
int orc_project(const orc_geom *g, const orc_opts *o, const double *x, double *b,
                int view_lo, int view_hi)
{
    const size_t npix = (size_t)g->nrows * g->ncols;
    const int nt = nthreads();
    double *sigma = (double *)malloc(npix * sizeof(double));
    double *part = (double *)calloc((size_t)nt * npix, sizeof(double));
    if (!sigma || !part) { free(sigma); free(part); return -1; }
    orc_pixel_scale_view(g, view_lo, o->scaling, sigma);
    int err = 0;
    for (int view = view_lo; view < view_hi; ++view) {
        if (g->frames && view != view_lo) orc_pixel_scale_view(g, view, o->scaling, sigma);
        memset(part, 0, (size_t)nt * npix * sizeof(double));
#pragma omp parallel
        {
            double *S = part + (size_t)thread_id() * npix;
            int32_t us[MAXW], vs[MAXW];
            double ws[MAXW];
#pragma omp for schedule(dynamic, 4)
            for (int col = 0; col < g->n1 * g->n2; ++col) {
                int i = col % g->n1, j = col / g->n1;
                for (int k = 0; k < g->n3; ++k) {
                    double mu = x[((size_t)k * g->n2 + j) * g->n1 + i];
                    if (mu == 0) continue;
                    int n = orc_voxel_weights(g, o, view, i, j, k, us, vs, ws, MAXW);
                    if (n < 0) { err = 1; continue; }
                    for (int q = 0; q < n; ++q)
                        S[(size_t)vs[q] * g->ncols + us[q]] += mu * ws[q];
                }
            }
        }
        double *out = b + (size_t)(view - view_lo) * npix;
        for (size_t p = 0; p < npix; ++p) {
            double acc = 0;
            for (int t = 0; t < nt; ++t) acc += part[(size_t)t * npix + p];
            out[p] = sigma[p] * acc;
        }
    }
    free(sigma);
    free(part);
    return err ? -2 : 0;
}

/* x = A^T b over views [view_lo, view_hi) for the voxels listed in idx (linear
 * indices k*n2*n1 + j*n1 + i); b holds those views only. */
int orc_backproject_voxels(const orc_geom *g, const orc_opts *o, const double *b,
                           int view_lo, int view_hi, int64_t nidx,
                           const int64_t *idx, double *out)
{
    const size_t npix = (size_t)g->nrows * g->ncols;
    /* pixel factors: one table, or one per view with per-view frames */
    const int nsig = g->frames ? view_hi - view_lo : 1;
    double *sigma = (double *)malloc((size_t)(nsig > 0 ? nsig : 1) * npix * sizeof(double));
    if (!sigma) return -1;
    for (int q = 0; q < nsig; ++q) orc_pixel_scale_view(g, view_lo + q, o->scaling, sigma + (size_t)q * npix);
    int err = 0;
#pragma omp parallel
    {
        int32_t us[MAXW], vs[MAXW];
        double ws[MAXW];
#pragma omp for schedule(dynamic, 16)
        for (int64_t q = 0; q < nidx; ++q) {
            int64_t lin = idx[q];
            int i = (int)(lin % g->n1), j = (int)((lin / g->n1) % g->n2);
            int k = (int)(lin / ((int64_t)g->n1 * g->n2));
            double acc = 0;
            for (int view = view_lo; view < view_hi; ++view) {
                int n = orc_voxel_weights(g, o, view, i, j, k, us, vs, ws, MAXW);
                if (n < 0) { err = 1; break; }
                const double *bv = b + (size_t)(view - view_lo) * npix;
                const double *sg = sigma + (g->frames ? (size_t)(view - view_lo) * npix : 0);
                for (int p = 0; p < n; ++p) {
                    size_t pix = (size_t)vs[p] * g->ncols + us[p];
                    double term = ws[p] * sg[pix] * bv[pix];
                    if (g_mutation == 6) term = ws[p] * sg[pix] * bv[(pix + 1) % npix];
                    acc += term;
                }
            }
            out[q] = acc;
        }
    }
    free(sigma);
    return err ? -2 : 0;
}

/* x = A^T b for every voxel */
int orc_backproject(const orc_geom *g, const orc_opts *o, const double *b,
                    double *x, int view_lo, int view_hi)
{
    int64_t n = (int64_t)g->n1 * g->n2 * g->n3;
    int64_t *idx = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (!idx) return -1;
    for (int64_t q = 0; q < n; ++q) idx[q] = q;
    int r = orc_backproject_voxels(g, o, b, view_lo, view_hi, n, idx, x);
    free(idx);
    return r;
}

int orc_num_threads(void) { return nthreads(); }

/* Thread count of the OpenMP loops (timing only; the results do not depend
 * on it: every output element is summed by one thread in a fixed order). */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
