/* Exact dense matvec with the scaled CFIE matrix, one entry at a time (oracle; test
 * infrastructure, never linked into the library).
 *
 * Section 3, eqs. (disc1) and (disc3) with plain weights and alpha = 1/2:
 *   A~_ii = 1/2,   A~_ij = sqrt(w_i) K(x_i, x_j) sqrt(w_j)  (i != j),
 *   K(x, y) = e^{ik rho} / (4 pi rho^3) [ (1 - ik rho) ((x - y) . n(y)) - i eta rho^2 ],
 * the combined-field kernel of eq. (comb_ref) (double layer minus i eta single layer),
 * rho = |x - y|. Each entry is formed from this closed form and summed in index order;
 * no entry is stored. The same arithmetic as the NumPy oracle, only compiled, so that
 * products with the full matrix at tens of thousands of unknowns take seconds.
 *
 * Layout: x, nrm are structure-of-arrays (3 * n doubles: all x, then all y, then all z);
 * w has n entries; v, y are interleaved complex (2 * n doubles). adjoint != 0 forms
 * y = A~^H v (conjugate transpose) instead of y = A~ v.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>

static const double PI_D = 3.14159265358979323846;

/* Entry A~[i, j]. The complex products are written out in real arithmetic:
 * e^{ik rho} = c + i s, and (1 - ik rho) dn - i eta rho^2 = dn + i q with
 * q = -(k rho dn + eta rho^2). */
static double complex entry(const double* x, const double* nrm, const double* sw, int64_t n,
                            double k, double eta, int64_t i, int64_t j)
{
    if (i == j) return 0.5;
    double dx = x[i] - x[j], dy = x[n + i] - x[n + j], dz = x[2 * n + i] - x[2 * n + j];
    double rho2 = dx * dx + dy * dy + dz * dz;
    double rho = sqrt(rho2);
    double dn = dx * nrm[j] + dy * nrm[n + j] + dz * nrm[2 * n + j];
    double c = cos(k * rho), s = sin(k * rho);
    double q = -(k * rho * dn + eta * rho2);
    double scale = sw[i] * sw[j] / (4.0 * PI_D * rho2 * rho);
    double re = (c * dn - s * q) * scale, im = (s * dn + c * q) * scale;
    return re + I * im;
}

void oracle_matvec(const double* x, const double* nrm, const double* sw, int64_t n, double k,
                   double eta, const double* v_in, double* y_out, int adjoint)
{
    const double complex* v = (const double complex*)v_in;
    double complex* y = (double complex*)y_out;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        double ar = 0.0, ai = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            double complex a = adjoint ? conj(entry(x, nrm, sw, n, k, eta, j, i)) : entry(x, nrm, sw, n, k, eta, i, j);
            double vr = creal(v[j]), vi = cimag(v[j]);
            ar += creal(a) * vr - cimag(a) * vi;
            ai += creal(a) * vi + cimag(a) * vr;
        }
        y[i] = ar + I * ai;
    }
}

/* Rows `rows[0..nr)` of A~ applied to v: y[t] = sum_j A~[rows[t], j] v[j]. */
void oracle_matvec_rows(const double* x, const double* nrm, const double* sw, int64_t n, double k,
                        double eta, const double* v_in, const int64_t* rows, int64_t nr, double* y_out)
{
    const double complex* v = (const double complex*)v_in;
    double complex* y = (double complex*)y_out;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t = 0; t < nr; ++t) {
        double ar = 0.0, ai = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            double complex a = entry(x, nrm, sw, n, k, eta, rows[t], j);
            double vr = creal(v[j]), vi = cimag(v[j]);
            ar += creal(a) * vr - cimag(a) * vi;
            ai += creal(a) * vi + cimag(a) * vr;
        }
        y[t] = ar + I * ai;
    }
}
