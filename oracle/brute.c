/* Brute-force FP64 sums for the oracle.  Test infrastructure only.
 *
 * A grid holds nx*ny*nz voxels stored [z][y][x].  Gaussian i has an index-frame centre
 * c[i] (3), conic C[i] (3x3, row-major, the inverse covariance in the grid's index frame),
 * amplitude amp[i] and an inclusive integer box lo[i]..hi[i] (x, y, z) that is used only
 * when nonempty[i] != 0.  The value of Gaussian i at voxel v is
 *     amp[i] * exp(-0.5 * (v - c)^T C (v - c))     when v lies in its box, else 0
 * (the paper's volumetric rendering, Eq. 7, truncated to the box).
 *
 * Sums run over Gaussians in ascending index.  No tiles, no binning, no reordering.
 */
#include <math.h>
#include <stdint.h>

static double gauss_value(const double* c, const double* C, double amp,
                          double x, double y, double z)
{
    const double d0 = x - c[0], d1 = y - c[1], d2 = z - c[2];
    const double q = d0 * (C[0] * d0 + C[1] * d1 + C[2] * d2)
                   + d1 * (C[3] * d0 + C[4] * d1 + C[5] * d2)
                   + d2 * (C[6] * d0 + C[7] * d1 + C[8] * d2);
    return amp * exp(-0.5 * q);
}

static int in_box(const int64_t* lo, const int64_t* hi, int64_t x, int64_t y, int64_t z)
{
    return x >= lo[0] && x <= hi[0] && y >= lo[1] && y <= hi[1] && z >= lo[2] && z <= hi[2];
}

/* out[z][y][x] = sum over every Gaussian i (ascending) of its value, if v is in its box. */
void oracle_render(int64_t nx, int64_t ny, int64_t nz, int64_t n, const double* c,
                   const double* C, const double* amp, const int64_t* lo, const int64_t* hi,
                   const uint8_t* nonempty, double* out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t z = 0; z < nz; ++z) {
        for (int64_t y = 0; y < ny; ++y) {
            for (int64_t x = 0; x < nx; ++x) {
                double acc = 0.0;
                for (int64_t i = 0; i < n; ++i) {
                    if (!nonempty[i] || !in_box(lo + 3 * i, hi + 3 * i, x, y, z)) continue;
                    acc += gauss_value(c + 3 * i, C + 9 * i, amp[i], (double)x, (double)y,
                                       (double)z);
                }
                out[(z * ny + y) * nx + x] = acc;
            }
        }
    }
}

/* The same sum at selected voxels pts[k] = (x, y, z). */
void oracle_render_points(int64_t npts, const int64_t* pts, int64_t n, const double* c,
                          const double* C, const double* amp, const int64_t* lo,
                          const int64_t* hi, const uint8_t* nonempty, double* out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < npts; ++k) {
        const int64_t x = pts[3 * k], y = pts[3 * k + 1], z = pts[3 * k + 2];
        double acc = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            if (!nonempty[i] || !in_box(lo + 3 * i, hi + 3 * i, x, y, z)) continue;
            acc += gauss_value(c + 3 * i, C + 9 * i, amp[i], (double)x, (double)y, (double)z);
        }
        out[k] = acc;
    }
}

/* The same sum as oracle_render, visiting each Gaussian's box instead of testing every
 * Gaussian at every voxel: plane z collects, in ascending i, the box rows of the Gaussians
 * whose box holds z.  Each voxel receives exactly the terms, and in exactly the order, of
 * oracle_render (starting from 0.0), so the results are identical; it costs the box volumes
 * instead of voxels x Gaussians.  out must be zeroed by the caller. */
void oracle_scatter_render(int64_t nx, int64_t ny, int64_t nz, int64_t n, const double* c,
                           const double* C, const double* amp, const int64_t* lo,
                           const int64_t* hi, const uint8_t* nonempty, double* out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t z = 0; z < nz; ++z) {
        for (int64_t i = 0; i < n; ++i) {
            if (!nonempty[i] || z < lo[3 * i + 2] || z > hi[3 * i + 2]) continue;
            for (int64_t y = lo[3 * i + 1]; y <= hi[3 * i + 1]; ++y)
                for (int64_t x = lo[3 * i]; x <= hi[3 * i]; ++x)
                    out[(z * ny + y) * nx + x] += gauss_value(c + 3 * i, C + 9 * i, amp[i],
                                                              (double)x, (double)y, (double)z);
        }
    }
}

/* For L = sum_v g[v] I[v]: per Gaussian, over the voxels of its box,
 *   d_amp[i]  = sum g * e            (e = exp(-q/2), w = amp * e)
 *   d_c[i]    = sum g * w * C (v - c)
 *   G_C[i]    = sum g * w * (-1/2) (v - c)(v - c)^T      (dL/dC, 3x3 row-major)     */
void oracle_partials(int64_t nx, int64_t ny, int64_t nz, int64_t n, const double* c,
                     const double* C, const double* amp, const int64_t* lo,
                     const int64_t* hi, const uint8_t* nonempty, const double* g,
                     double* d_amp, double* d_c, double* G_C)
{
    (void)nz;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        double s_amp = 0.0, s_c[3] = {0, 0, 0}, s_C[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        if (nonempty[i]) {
            const double* ci = c + 3 * i;
            const double* Ci = C + 9 * i;
            for (int64_t z = lo[3 * i + 2]; z <= hi[3 * i + 2]; ++z)
                for (int64_t y = lo[3 * i + 1]; y <= hi[3 * i + 1]; ++y)
                    for (int64_t x = lo[3 * i]; x <= hi[3 * i]; ++x) {
                        const double gv = g[(z * ny + y) * nx + x];
                        const double d[3] = {(double)x - ci[0], (double)y - ci[1],
                                             (double)z - ci[2]};
                        const double e = gauss_value(ci, Ci, 1.0, (double)x, (double)y,
                                                     (double)z);
                        const double gw = gv * amp[i] * e;
                        s_amp += gv * e;
                        for (int a = 0; a < 3; ++a) {
                            s_c[a] += gw * (Ci[3 * a] * d[0] + Ci[3 * a + 1] * d[1]
                                            + Ci[3 * a + 2] * d[2]);
                            for (int b = 0; b < 3; ++b) s_C[3 * a + b] += -0.5 * gw * d[a] * d[b];
                        }
                    }
        }
        d_amp[i] = s_amp;
        for (int a = 0; a < 3; ++a) d_c[3 * i + a] = s_c[a];
        for (int a = 0; a < 9; ++a) G_C[9 * i + a] = s_C[a];
    }
}

/* The paper's cell-neighbourhood query (Sec. 3.3.1, Eqs. 4-6) on any grid: voxel v takes
 * Gaussian i when valid[i] != 0 and, on every world axis a, the cell of v's world position
 * vcell[v][a] lies within radius of the cell of the Gaussian's mean gcell[i][a].  No box. */
static int in_block(const int64_t* vc, const int64_t* gc, int64_t radius)
{
    for (int a = 0; a < 3; ++a) {
        const int64_t d = vc[a] - gc[a];
        if (d < -radius || d > radius) return 0;
    }
    return 1;
}

/* oracle_render with the block test in place of the box test. */
void oracle_render_cells(int64_t nx, int64_t ny, int64_t nz, int64_t n, const double* c,
                         const double* C, const double* amp, const int64_t* vcell,
                         const int64_t* gcell, const uint8_t* valid, int64_t radius,
                         double* out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t z = 0; z < nz; ++z) {
        for (int64_t y = 0; y < ny; ++y) {
            for (int64_t x = 0; x < nx; ++x) {
                const int64_t v = (z * ny + y) * nx + x;
                double acc = 0.0;
                for (int64_t i = 0; i < n; ++i) {
                    if (!valid[i] || !in_block(vcell + 3 * v, gcell + 3 * i, radius)) continue;
                    acc += gauss_value(c + 3 * i, C + 9 * i, amp[i], (double)x, (double)y,
                                       (double)z);
                }
                out[v] = acc;
            }
        }
    }
}

/* oracle_render_points with the block test in place of the box test: pcell[k] is the cell
 * of point k's world position. */
void oracle_render_points_cells(int64_t npts, const int64_t* pts, const int64_t* pcell,
                                int64_t n, const double* c, const double* C, const double* amp,
                                const int64_t* gcell, const uint8_t* valid, int64_t radius,
                                double* out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < npts; ++k) {
        const int64_t x = pts[3 * k], y = pts[3 * k + 1], z = pts[3 * k + 2];
        double acc = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            if (!valid[i] || !in_block(pcell + 3 * k, gcell + 3 * i, radius)) continue;
            acc += gauss_value(c + 3 * i, C + 9 * i, amp[i], (double)x, (double)y, (double)z);
        }
        out[k] = acc;
    }
}

/* oracle_partials over the voxels the block test gives each Gaussian. */
void oracle_partials_cells(int64_t nx, int64_t ny, int64_t nz, int64_t n, const double* c,
                           const double* C, const double* amp, const int64_t* vcell,
                           const int64_t* gcell, const uint8_t* valid, int64_t radius,
                           const double* g, double* d_amp, double* d_c, double* G_C)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        double s_amp = 0.0, s_c[3] = {0, 0, 0}, s_C[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        const double* ci = c + 3 * i;
        const double* Ci = C + 9 * i;
        for (int64_t z = 0; valid[i] && z < nz; ++z)
            for (int64_t y = 0; y < ny; ++y)
                for (int64_t x = 0; x < nx; ++x) {
                    const int64_t v = (z * ny + y) * nx + x;
                    if (!in_block(vcell + 3 * v, gcell + 3 * i, radius)) continue;
                    const double gv = g[v];
                    const double d[3] = {(double)x - ci[0], (double)y - ci[1], (double)z - ci[2]};
                    const double e = gauss_value(ci, Ci, 1.0, (double)x, (double)y, (double)z);
                    const double gw = gv * amp[i] * e;
                    s_amp += gv * e;
                    for (int a = 0; a < 3; ++a) {
                        s_c[a] += gw * (Ci[3 * a] * d[0] + Ci[3 * a + 1] * d[1]
                                        + Ci[3 * a + 2] * d[2]);
                        for (int b = 0; b < 3; ++b) s_C[3 * a + b] += -0.5 * gw * d[a] * d[b];
                    }
                }
        d_amp[i] = s_amp;
        for (int a = 0; a < 3; ++a) d_c[3 * i + a] = s_c[a];
        for (int a = 0; a < 9; ++a) G_C[9 * i + a] = s_C[a];
    }
}

#ifdef _OPENMP
#include <omp.h>
#endif
/* Threads the OpenMP loops above use. */
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Set the thread count of the loops above (k <= 0 leaves it unchanged). */
void oracle_set_threads(int k)
{
#ifdef _OPENMP
    if (k > 0) omp_set_num_threads(k);
#else
    (void)k;
#endif
}
