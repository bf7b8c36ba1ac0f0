/*
 * FP64 reference: running integral of the irreversible two-tissue tissue curve, in closed form.
 *
 * TEST INFRASTRUCTURE ONLY.  This file belongs to the CPU oracle that the tests use to check
 * the HIP library; nothing in the library links or calls it.
 *
 * Model (Sec. II-C; the time integrals of the kinetic model are analytic): with a = k2 + k3 the
 * impulse response of the tissue is K1 (k3 + k2 e^{-a t}) / a, so
 *
 *     int_0^T C_T = K1 [ alpha P2(T) + (1 - alpha) I(T) ],   alpha = k3 / a,
 *
 * where P1 = int_0^T Cp, P2 = int_0^T P1 (voxel independent, passed in), G = Cp (*) e^{-a t}
 * and I = int_0^T G = (P1 - G) / a (from G' = Cp - a G).  The derivatives also need
 * A4 = Cp (*) (t e^{-a t}):
 *
 *     d/dK1 = alpha P2 + (1 - alpha) I,
 *     d/dk2 = K1 [ -(k3 / a^2) (P2 - I) + (k2 / a^2) (A4 - I) ],
 *     d/dk3 = K1 [  (k2 / a^2) (P2 - I) + (k2 / a^2) (A4 - I) ].
 *
 * The plasma input is a sum of components c t^n e^{l t} (n = 0 or 1).  Per component, with
 * b = l + a, both convolutions reduce to moments m_k(z) = int_0^1 s^k e^{z s} ds of a
 * non-positive exponent z:
 *   b <= 0 (substitute s = T sigma):  G = e^{-aT} T^{n+1} m_n(bT),
 *                                     A4 = e^{-aT} T^{n+2} (m_n - m_{n+1})(bT);
 *   b > 0  (substitute u = T - s):    n = 0: G = e^{lT} T m_0(-bT),        A4 = e^{lT} T^2 m_1(-bT);
 *                                     n = 1: G = e^{lT} T^2 (m_0 - m_1),   A4 = e^{lT} T^3 (m_1 - m_2).
 * m_k is its power series sum_j z^j / (j! (j + k + 1)) for |z| < 1 (26 terms) and the recursion
 * m_0 = expm1(z) / z, m_k = (e^z - k m_{k-1}) / z otherwise.
 */
#include <math.h>
#include <stdint.h>

/* m_k(z) for k = 0..kmax (kmax <= 3). */
static void moments(double z, int kmax, double* m) {
    if (fabs(z) < 1.0) {
        double term = 1.0; /* z^j / j! */
        for (int k = 0; k <= kmax; ++k) m[k] = 0.0;
        for (int j = 0; j < 26; ++j) {
            for (int k = 0; k <= kmax; ++k) m[k] += term / (double)(j + k + 1);
            term *= z / (double)(j + 1);
        }
        return;
    }
    const double ez = exp(z);
    m[0] = expm1(z) / z;
    for (int k = 1; k <= kmax; ++k) m[k] = (ez - (double)k * m[k - 1]) / z;
}

/* For n voxels (params row-major (K1, k2, k3), k2 + k3 > 0) and nT times T with the input
 * integrals P1, P2 there: C[v * nT + t] = int_0^T C_T and, if D is not NULL,
 * D[(v * nT + t) * 3 + p] = its derivative by parameter p.  comp holds ncomp input components
 * as (c, l, n) triples. */
void orc_tissue_integrals(int64_t n, const double* params, int32_t nT, const double* T, const double* P1,
                          const double* P2, int32_t ncomp, const double* comp, double* C, double* D) {
#pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < n; ++v) {
        const double K1 = params[3 * v], k2 = params[3 * v + 1], k3 = params[3 * v + 2];
        const double a = k2 + k3, alpha = k3 / a, a2 = a * a;
        for (int32_t t = 0; t < nT; ++t) {
            const double Tt = T[t];
            double G = 0.0, A4 = 0.0;
            for (int32_t i = 0; i < ncomp; ++i) {
                const double c = comp[3 * i], l = comp[3 * i + 1];
                const int pw = (int)comp[3 * i + 2];
                const double b = l + a;
                double m[4], g, a4;
                if (b <= 0.0) {
                    moments(b * Tt, pw + 1, m);
                    const double e = exp(-a * Tt), tp = pow(Tt, pw + 1);
                    g = e * tp * m[pw];
                    a4 = e * tp * Tt * (m[pw] - m[pw + 1]);
                } else {
                    moments(-b * Tt, 2, m);
                    const double e = exp(l * Tt);
                    if (pw == 0) {
                        g = e * Tt * m[0];
                        a4 = e * Tt * Tt * m[1];
                    } else {
                        g = e * Tt * Tt * (m[0] - m[1]);
                        a4 = e * Tt * Tt * Tt * (m[1] - m[2]);
                    }
                }
                G += c * g;
                A4 += c * a4;
            }
            const double I = (P1[t] - G) / a;
            const double dK1 = alpha * P2[t] + (1.0 - alpha) * I;
            C[v * nT + t] = K1 * dK1;
            if (D) {
                double* d = D + (v * nT + t) * 3;
                d[0] = dK1;
                d[1] = K1 * (-(k3 / a2) * (P2[t] - I) + (k2 / a2) * (A4 - I));
                d[2] = K1 * ((k2 / a2) * (P2[t] - I) + (k2 / a2) * (A4 - I));
            }
        }
    }
}
