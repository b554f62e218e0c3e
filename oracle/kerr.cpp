/*
 * Kerr geometry in Kerr-Schild coordinates (t, r, theta, phi), G = c = M = 1.
 * Test infrastructure only (CPU oracle).
 *
 * The paper (Sec. 2.1) integrates null geodesics of the black-hole spacetime;
 * it does not name a coordinate system.  Reading: horizon-penetrating
 * Kerr-Schild coordinates, metric written out below, inverse obtained by
 * plain Gauss-Jordan elimination, Christoffel symbols from the textbook
 * definition with analytic first derivatives of the metric.
 *
 * A mass factor m multiplies the mass term: m = 1 is Kerr, m = 0 is flat
 * space in spheroidal coordinates (used by the flat-space tests).
 */
#include <cmath>
#include <cstring>
#include "oracle_internal.h"

namespace orc {

/* g_{mu nu}.  With Sigma = r^2 + a^2 cos^2, f = 2 m r / Sigma:
 * g_tt = -(1-f), g_tr = f, g_tph = -a f sin^2, g_rr = 1+f,
 * g_rph = -a sin^2 (1+f), g_thth = Sigma, g_phph = sin^2 (Sigma + a^2 sin^2 (1+f)). */
void metric(double a, double m, double r, double th, Mat4 g) {
    double s = std::sin(th), c = std::cos(th);
    double s2 = s * s;
    double Sig = r * r + a * a * c * c;
    double f = 2.0 * m * r / Sig;
    std::memset(g, 0, sizeof(Mat4));
    g[0][0] = -(1.0 - f);
    g[0][1] = g[1][0] = f;
    g[0][3] = g[3][0] = -a * f * s2;
    g[1][1] = 1.0 + f;
    g[1][3] = g[3][1] = -a * s2 * (1.0 + f);
    g[2][2] = Sig;
    g[3][3] = s2 * (Sig + a * a * s2 * (1.0 + f));
}

/* dg[k][mu][nu] = d g_{mu nu} / d x^k.  Only k = r (1) and k = theta (2)
 * are non-zero (stationary, axisymmetric). */
void metric_derivs(double a, double m, double r, double th, double dg[4][4][4]) {
    std::memset(dg, 0, sizeof(double) * 64);
    double s = std::sin(th), c = std::cos(th);
    double s2 = s * s, sc = s * c;
    double Sig = r * r + a * a * c * c;
    double Sig_r = 2.0 * r;
    double Sig_t = -2.0 * a * a * sc;
    double f = 2.0 * m * r / Sig;
    double f_r = 2.0 * m / Sig - 2.0 * m * r * Sig_r / (Sig * Sig);
    double f_t = -2.0 * m * r * Sig_t / (Sig * Sig);
    double s2_t = 2.0 * sc;

    /* radial derivatives */
    double (*R)[4] = dg[1];
    R[0][0] = f_r;
    R[0][1] = R[1][0] = f_r;
    R[0][3] = R[3][0] = -a * f_r * s2;
    R[1][1] = f_r;
    R[1][3] = R[3][1] = -a * s2 * f_r;
    R[2][2] = Sig_r;
    R[3][3] = s2 * (Sig_r + a * a * s2 * f_r);

    /* polar derivatives */
    double (*T)[4] = dg[2];
    T[0][0] = f_t;
    T[0][1] = T[1][0] = f_t;
    T[0][3] = T[3][0] = -a * (f_t * s2 + f * s2_t);
    T[1][1] = f_t;
    T[1][3] = T[3][1] = -a * (s2_t * (1.0 + f) + s2 * f_t);
    T[2][2] = Sig_t;
    T[3][3] = s2_t * (Sig + a * a * s2 * (1.0 + f))
            + s2 * (Sig_t + a * a * (s2_t * (1.0 + f) + s2 * f_t));
}

/* Gauss-Jordan inversion with partial pivoting.  Returns 0 on success. */
int invert4(const Mat4 A, Mat4 Ainv) {
    double M[4][8];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            M[i][j] = A[i][j];
            M[i][j + 4] = (i == j) ? 1.0 : 0.0;
        }
    for (int col = 0; col < 4; ++col) {
        int piv = col;
        for (int i = col + 1; i < 4; ++i)
            if (std::fabs(M[i][col]) > std::fabs(M[piv][col])) piv = i;
        if (M[piv][col] == 0.0) return -1;
        if (piv != col)
            for (int j = 0; j < 8; ++j) std::swap(M[piv][j], M[col][j]);
        double p = M[col][col];
        for (int j = 0; j < 8; ++j) M[col][j] /= p;
        for (int i = 0; i < 4; ++i) {
            if (i == col) continue;
            double fac = M[i][col];
            for (int j = 0; j < 8; ++j) M[i][j] -= fac * M[col][j];
        }
    }
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) Ainv[i][j] = M[i][j + 4];
    return 0;
}

/* Gamma^mu_{al be} = 1/2 g^{mu nu} (d_al g_{nu be} + d_be g_{nu al} - d_nu g_{al be}). */
void christoffel(double a, double m, double r, double th, double G[4][4][4]) {
    Mat4 g, gi;
    double dg[4][4][4];
    metric(a, m, r, th, g);
    invert4(g, gi);
    metric_derivs(a, m, r, th, dg);
    for (int mu = 0; mu < 4; ++mu)
        for (int al = 0; al < 4; ++al)
            for (int be = 0; be < 4; ++be) {
                double s = 0.0;
                for (int nu = 0; nu < 4; ++nu)
                    s += gi[mu][nu] * (dg[al][nu][be] + dg[be][nu][al] - dg[nu][al][be]);
                G[mu][al][be] = 0.5 * s;
            }
}

/* Outer horizon r_+ = m + sqrt(m^2 - a^2) (m = 1 for Kerr). */
double horizon(double a, double m) {
    if (m == 0.0) return 0.0;
    return m + std::sqrt(m * m - a * a);
}

/* Innermost stable circular orbit of Kerr (Bardeen, Press & Teukolsky 1972);
 * prograde for a > 0. */
double isco(double a) {
    double aa = std::fabs(a);
    double z1 = 1.0 + std::cbrt(1.0 - aa * aa) * (std::cbrt(1.0 + aa) + std::cbrt(1.0 - aa));
    double z2 = std::sqrt(3.0 * aa * aa + z1 * z1);
    double sgn = (a >= 0.0) ? 1.0 : -1.0;
    return 3.0 + z2 - sgn * std::sqrt((3.0 - z1) * (3.0 + z1 + 2.0 * z2));
}

double dot(const Mat4 g, const double x[4], const double y[4]) {
    double s = 0.0;
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) s += g[i][j] * x[i] * y[j];
    return s;
}

void lower(const Mat4 g, const double x[4], double xl[4]) {
    for (int i = 0; i < 4; ++i) {
        double s = 0.0;
        for (int j = 0; j < 4; ++j) s += g[i][j] * x[j];
        xl[i] = s;
    }
}

}  // namespace orc
