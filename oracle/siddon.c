/*
 * FP64 reference: exact ray/pixel intersection lengths for a 2D parallel-beam geometry.
 *
 * TEST INFRASTRUCTURE ONLY.  This file belongs to the CPU oracle that the tests use to check
 * the HIP library; nothing in the library links or calls it.
 *
 * The system matrix element p_vd (Eq. 2) is the length, in mm, of the intersection of ray d
 * with the square of pixel v.  It is computed with Siddon's algorithm (1985): the ray is a
 * parametric segment p(alpha) = p1 + alpha (p2 - p1); the parameters at which it crosses the
 * vertical and horizontal grid lines inside the image are merged in increasing order; each
 * pair of consecutive parameters bounds one segment whose midpoint names the pixel and whose
 * parameter difference times the segment length is the intersection length.
 *
 * Geometry: pixels are squares of side h; pixel (i, j) spans
 * [X0 + i h, X0 + (i+1) h) x [Y0 + j h, Y0 + (j+1) h) with X0 = -nx h / 2, Y0 = -ny h / 2
 * (half-open, so a ray lying on a grid line belongs to the higher index).  Ray (a, b) is the
 * line x cos(t_a) + y sin(t_a) = u_b with t_a = ang0 + a pi / n_ang and
 * u_b = (b - (n_bin - 1) / 2) du.  Rows of the matrix are ordered a-major, then b.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t nx, ny;
    double h;      /* pixel side, mm */
    int32_t n_ang, n_bin;
    double du;     /* bin width, mm */
    double ang0;   /* first angle, rad */
} orc_geom2d;

/* cos and sin of the ray normal of angle a, snapped exactly at multiples of pi/2. */
void orc_ray_cos_sin(const orc_geom2d* g, int32_t a, double* c, double* s) {
    double t = g->ang0 + (double)a * M_PI / (double)g->n_ang;
    double cc = cos(t), ss = sin(t);
    if (fabs(cc) < 1e-12) { cc = 0.0; ss = ss > 0 ? 1.0 : -1.0; }
    if (fabs(ss) < 1e-12) { ss = 0.0; cc = cc > 0 ? 1.0 : -1.0; }
    *c = cc;
    *s = ss;
}

static int cmp_double(const void* pa, const void* pb) {
    double a = *(const double*)pa, b = *(const double*)pb;
    return (a > b) - (a < b);
}

/* Intersections of the line x c + y s = u with the image grid.  Writes at most `cap` pairs
 * (pixel index j*nx+i, length) and returns how many pairs the ray has.  `work` must hold
 * nx + ny + 4 doubles. */
int32_t orc_siddon_line(const orc_geom2d* g, double c, double s, double u,
                        int64_t* idx, double* len, int32_t cap, double* work) {
    const double h = g->h;
    const double X0 = -0.5 * g->nx * h, Y0 = -0.5 * g->ny * h;
    const double X1 = X0 + g->nx * h, Y1 = Y0 + g->ny * h;
    const double R = h * (double)(g->nx + g->ny);  /* half-length, beyond the image */
    /* direction (-s, c), foot point u (c, s) */
    const double p1x = u * c + R * s, p1y = u * s - R * c;
    const double dx = -2.0 * R * s, dy = 2.0 * R * c;
    const double L = 2.0 * R;

    double amin = 0.0, amax = 1.0;
    if (dx != 0.0) {
        double a0 = (X0 - p1x) / dx, a1 = (X1 - p1x) / dx;
        amin = fmax(amin, fmin(a0, a1));
        amax = fmin(amax, fmax(a0, a1));
    } else if (!(p1x >= X0 && p1x < X1)) {
        return 0;
    }
    if (dy != 0.0) {
        double a0 = (Y0 - p1y) / dy, a1 = (Y1 - p1y) / dy;
        amin = fmax(amin, fmin(a0, a1));
        amax = fmin(amax, fmax(a0, a1));
    } else if (!(p1y >= Y0 && p1y < Y1)) {
        return 0;
    }
    if (!(amax > amin)) return 0;

    int32_t n = 0;
    work[n++] = amin;
    work[n++] = amax;
    if (dx != 0.0) {
        for (int32_t i = 0; i <= g->nx; ++i) {
            double a = (X0 + i * h - p1x) / dx;
            if (a > amin && a < amax) work[n++] = a;
        }
    }
    if (dy != 0.0) {
        for (int32_t j = 0; j <= g->ny; ++j) {
            double a = (Y0 + j * h - p1y) / dy;
            if (a > amin && a < amax) work[n++] = a;
        }
    }
    qsort(work, (size_t)n, sizeof(double), cmp_double);

    int32_t m = 0;
    for (int32_t k = 0; k + 1 < n; ++k) {
        double a0 = work[k], a1 = work[k + 1];
        if (!(a1 > a0)) continue;
        double am = 0.5 * (a0 + a1);
        double px = p1x + am * dx, py = p1y + am * dy;
        int64_t i = (int64_t)floor((px - X0) / h);
        int64_t j = (int64_t)floor((py - Y0) / h);
        if (i < 0 || i >= g->nx || j < 0 || j >= g->ny) continue;
        if (m < cap) {
            idx[m] = j * g->nx + i;
            len[m] = (a1 - a0) * L;
        }
        ++m;
    }
    return m;
}

static double bin_centre(const orc_geom2d* g, int32_t b) {
    return ((double)b - 0.5 * (double)(g->n_bin - 1)) * g->du;
}

/* Number of nonzeros per row (row = a * n_bin + b); row_ptr has n_ang*n_bin+1 entries. */
int64_t orc_csr_count(const orc_geom2d* g, int64_t* row_ptr) {
    const int64_t n_rows = (int64_t)g->n_ang * g->n_bin;
    row_ptr[0] = 0;
#pragma omp parallel
    {
        double* work = (double*)malloc(sizeof(double) * (size_t)(g->nx + g->ny + 4));
#pragma omp for schedule(dynamic, 64)
        for (int64_t r = 0; r < n_rows; ++r) {
            int32_t a = (int32_t)(r / g->n_bin), b = (int32_t)(r % g->n_bin);
            double c, s;
            orc_ray_cos_sin(g, a, &c, &s);
            row_ptr[r + 1] = orc_siddon_line(g, c, s, bin_centre(g, b), NULL, NULL, 0, work);
        }
        free(work);
    }
    for (int64_t r = 0; r < n_rows; ++r) row_ptr[r + 1] += row_ptr[r];
    return row_ptr[n_rows];
}

/* Fill column indices and lengths of the CSR matrix whose row_ptr came from orc_csr_count. */
void orc_csr_fill(const orc_geom2d* g, const int64_t* row_ptr, int64_t* col, double* val) {
    const int64_t n_rows = (int64_t)g->n_ang * g->n_bin;
#pragma omp parallel
    {
        double* work = (double*)malloc(sizeof(double) * (size_t)(g->nx + g->ny + 4));
#pragma omp for schedule(dynamic, 64)
        for (int64_t r = 0; r < n_rows; ++r) {
            int32_t a = (int32_t)(r / g->n_bin), b = (int32_t)(r % g->n_bin);
            double c, s;
            orc_ray_cos_sin(g, a, &c, &s);
            int32_t cap = (int32_t)(row_ptr[r + 1] - row_ptr[r]);
            orc_siddon_line(g, c, s, bin_centre(g, b), col + row_ptr[r], val + row_ptr[r], cap, work);
        }
        free(work);
    }
}
