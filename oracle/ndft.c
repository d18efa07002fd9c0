/*
 * Direct NUDFT oracle in FP64 (test infrastructure only).
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * load this library.  It shares no code with the GPU library.
 *
 * It evaluates the exact non-uniform DFT of the system model (Sec. II-B,
 * eq. (e,ndft)):
 *
 *     a_ij = exp(-i omega_i . r_j),   y = A x,   x_hat = A^H y,
 *
 * where r_j is the centre of voxel j on the Cartesian grid.  Reading of the
 * paper's silent points (they fix the operator, so they are stated here):
 *   - coordinate of index j on an axis of length n is r = j - floor(n/2)
 *     (integer voxel units, omega in radians per voxel);
 *   - images are row-major, axis 0 slowest; omega[m*D + d] pairs with axis d;
 *   - no normalisation; forward uses exp(-i ...), adjoint exp(+i ...).
 *
 * Optional weight: with wdim >= 0 the image is multiplied by the coordinate
 * r^[wdim] inside the sum, which is the operand A(x (.) r^[d]) of the
 * omega-Jacobians (Sec. II-C eq. (e,Ax), Sec. II-D eq. (e,A'y)).
 *
 * exp(-i omega . r) is the product over axes of exp(-i omega_d r_d); every
 * factor is a direct libm cos/sin call (no recurrences), and the sum is taken
 * axis by axis.  Complex numbers are interleaved (re, im) doubles.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

static double coord(int64_t j, int64_t n) { return (double)(j - n / 2); }

/* Pad the shape to three axes (missing leading axes have length 1). */
static void shape3(int D, const int64_t *N, int64_t n3[3]) {
    n3[0] = n3[1] = n3[2] = 1;
    for (int d = 0; d < D; ++d) n3[3 - D + d] = N[d];
}

int ndft_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * y[c*M + m] = sum_j w(j) x[c*Ntot + j] exp(-i omega_m . r_j)  for c < nch,
 * w(j) = r^[wdim]_j if wdim >= 0, else 1.   Rows m may be restricted to the
 * list rows[0..nrows) (rows == NULL: all M rows); y then holds nrows rows.
 */
int ndft_forward(int D, const int64_t *N, int64_t M, const double *omega, int nch,
                 const double *x, int wdim, const int64_t *rows, int64_t nrows,
                 double *y) {
    if (D < 1 || D > 3 || nch < 1) return -1;
    int64_t n3[3];
    shape3(D, N, n3);
    const int64_t Ntot = n3[0] * n3[1] * n3[2];
    const int64_t R = rows ? nrows : M;
    const int wax = wdim >= 0 ? 3 - D + wdim : -1; /* weighted axis in padded shape */

#pragma omp parallel
    {
        double *e[3];
        for (int a = 0; a < 3; ++a) e[a] = (double *)malloc(sizeof(double) * 2 * n3[a]);
#pragma omp for schedule(dynamic, 16)
        for (int64_t q = 0; q < R; ++q) {
            const int64_t m = rows ? rows[q] : q;
            for (int a = 0; a < 3; ++a) {
                const int d = a - (3 - D);
                const double om = d >= 0 ? omega[m * D + d] : 0.0;
                for (int64_t j = 0; j < n3[a]; ++j) {
                    const double ph = om * (d >= 0 ? coord(j, n3[a]) : 0.0);
                    const double w = (a == wax) ? coord(j, n3[a]) : 1.0;
                    e[a][2 * j] = w * cos(ph);
                    e[a][2 * j + 1] = -w * sin(ph);
                }
            }
            for (int c = 0; c < nch; ++c) {
                const double *xc = x + 2 * c * Ntot;
                double s0r = 0.0, s0i = 0.0;
                for (int64_t j0 = 0; j0 < n3[0]; ++j0) {
                    double s1r = 0.0, s1i = 0.0;
                    for (int64_t j1 = 0; j1 < n3[1]; ++j1) {
                        const double *row = xc + 2 * (j0 * n3[1] + j1) * n3[2];
                        double s2r = 0.0, s2i = 0.0;
                        for (int64_t j2 = 0; j2 < n3[2]; ++j2) {
                            const double er = e[2][2 * j2], ei = e[2][2 * j2 + 1];
                            const double xr = row[2 * j2], xi = row[2 * j2 + 1];
                            s2r += er * xr - ei * xi;
                            s2i += er * xi + ei * xr;
                        }
                        const double er = e[1][2 * j1], ei = e[1][2 * j1 + 1];
                        s1r += er * s2r - ei * s2i;
                        s1i += er * s2i + ei * s2r;
                    }
                    const double er = e[0][2 * j0], ei = e[0][2 * j0 + 1];
                    s0r += er * s1r - ei * s1i;
                    s0i += er * s1i + ei * s1r;
                }
                y[2 * (c * R + q)] = s0r;
                y[2 * (c * R + q) + 1] = s0i;
            }
        }
        for (int a = 0; a < 3; ++a) free(e[a]);
    }
    return 0;
}

/*
 * x[c*Ntot + j] = w(j) sum_m y[c*M + m] exp(+i omega_m . r_j)  for c < nch.
 * Pixels may be restricted to the flat indices pix[0..npix) (pix == NULL:
 * all pixels); x then holds npix values per channel.
 */
int ndft_adjoint(int D, const int64_t *N, int64_t M, const double *omega, int nch,
                 const double *y, int wdim, const int64_t *pix, int64_t npix,
                 double *x) {
    if (D < 1 || D > 3 || nch < 1) return -1;
    int64_t n3[3];
    shape3(D, N, n3);
    const int64_t Ntot = n3[0] * n3[1] * n3[2];
    const int64_t P = pix ? npix : Ntot;
    const int off = 3 - D;

#pragma omp parallel
    {
        double *acc = (double *)malloc(sizeof(double) * 2 * nch);
#pragma omp for schedule(dynamic, 4)
        for (int64_t q = 0; q < P; ++q) {
            const int64_t j = pix ? pix[q] : q;
            int64_t jj[3];
            jj[2] = j % n3[2];
            jj[1] = (j / n3[2]) % n3[1];
            jj[0] = j / (n3[1] * n3[2]);
            double r[3];
            for (int a = 0; a < 3; ++a) r[a] = coord(jj[a], n3[a]);
            const double w = wdim >= 0 ? r[off + wdim] : 1.0;
            memset(acc, 0, sizeof(double) * 2 * nch);
            for (int64_t m = 0; m < M; ++m) {
                /* exp(+i sum_d omega_d r_d) as a product of per-axis factors */
                double pr = 1.0, pi = 0.0;
                for (int d = 0; d < D; ++d) {
                    const double ph = omega[m * D + d] * r[off + d];
                    const double cr = cos(ph), ci = sin(ph);
                    const double tr = pr * cr - pi * ci;
                    pi = pr * ci + pi * cr;
                    pr = tr;
                }
                for (int c = 0; c < nch; ++c) {
                    const double yr = y[2 * (c * M + m)], yi = y[2 * (c * M + m) + 1];
                    acc[2 * c] += yr * pr - yi * pi;
                    acc[2 * c + 1] += yr * pi + yi * pr;
                }
            }
            for (int c = 0; c < nch; ++c) {
                x[2 * (c * P + q)] = w * acc[2 * c];
                x[2 * (c * P + q) + 1] = w * acc[2 * c + 1];
            }
        }
        free(acc);
    }
    return 0;
}

/*
 * Forward sum for an image that is zero outside the listed voxels:
 *   y[c*M + m] = sum_k x[c*npix + k] exp(-i omega_m . r_{pix[k]})   for c < nch,
 * i.e. eq. (e,ndft) with the zero terms left out.  The per-axis factors
 * exp(-i omega_{m,d} r) are direct libm calls for every coordinate of the
 * axis, as in ndft_forward; each listed voxel multiplies its D factors.
 * Used for problems whose image has too many voxels for the dense sum.
 */
int ndft_forward_sparse(int D, const int64_t *N, int64_t M, const double *omega, int nch,
                        const int64_t *pix, int64_t npix, const double *x, double *y) {
    if (D < 1 || D > 3 || nch < 1 || npix < 0) return -1;
    int64_t n3[3];
    shape3(D, N, n3);
    const int off = 3 - D;
    int64_t *jj = (int64_t *)malloc(sizeof(int64_t) * 3 * (npix > 0 ? npix : 1));
    for (int64_t k = 0; k < npix; ++k) {
        const int64_t j = pix[k];
        jj[3 * k + 2] = j % n3[2];
        jj[3 * k + 1] = (j / n3[2]) % n3[1];
        jj[3 * k] = j / (n3[1] * n3[2]);
    }
#pragma omp parallel
    {
        double *e[3];
        for (int a = 0; a < 3; ++a) e[a] = (double *)malloc(sizeof(double) * 2 * n3[a]);
#pragma omp for schedule(dynamic, 256)
        for (int64_t m = 0; m < M; ++m) {
            for (int a = 0; a < 3; ++a) {
                const int d = a - off;
                const double om = d >= 0 ? omega[m * D + d] : 0.0;
                for (int64_t j = 0; j < n3[a]; ++j) {
                    const double ph = om * (d >= 0 ? coord(j, n3[a]) : 0.0);
                    e[a][2 * j] = cos(ph);
                    e[a][2 * j + 1] = -sin(ph);
                }
            }
            for (int c = 0; c < nch; ++c) {
                const double *xc = x + 2 * c * npix;
                double sr = 0.0, si = 0.0;
                for (int64_t k = 0; k < npix; ++k) {
                    /* product of the three axis factors */
                    const double *f0 = e[0] + 2 * jj[3 * k], *f1 = e[1] + 2 * jj[3 * k + 1],
                                 *f2 = e[2] + 2 * jj[3 * k + 2];
                    const double ar = f0[0] * f1[0] - f0[1] * f1[1];
                    const double ai = f0[0] * f1[1] + f0[1] * f1[0];
                    const double pr = ar * f2[0] - ai * f2[1];
                    const double pi = ar * f2[1] + ai * f2[0];
                    const double xr = xc[2 * k], xi = xc[2 * k + 1];
                    sr += pr * xr - pi * xi;
                    si += pr * xi + pi * xr;
                }
                y[2 * (c * M + m)] = sr;
                y[2 * (c * M + m) + 1] = si;
            }
        }
        for (int a = 0; a < 3; ++a) free(e[a]);
    }
    free(jj);
    return 0;
}
