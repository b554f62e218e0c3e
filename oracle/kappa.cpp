/*
 * Synchrotron coefficients of a kappa electron distribution (and, for the
 * checks, of a Maxwell-Juttner one) by numerical integration over the
 * Lorentz factor.  Test infrastructure only (CPU oracle).
 *
 * Sec. 2.1 names the electron distribution among the model inputs and the
 * conclusions (Sec. 4) name nonthermal electrons as the next step; the paper
 * gives no formulae, so the method is written out from the standard theory:
 *
 *  - distribution (isotropic in pitch angle, normalised to one electron):
 *      kappa: N(g) = A g sqrt(g^2-1) (1 + (g-1)/(kappa w))^-(kappa+1)
 *      thermal: N(g) = A g sqrt(g^2-1) exp(-(g-1)/w)   (w = Theta_e)
 *    the width w plays the part of Theta_e; kappa -> infinity gives the
 *    thermal form.
 *  - emission of one ultrarelativistic electron seen at angle theta to the
 *    field (electrons with pitch angle theta dominate), per steradian:
 *      I: c0 F(Xg), Q: c0 G(Xg), V: c0 (4/3) (cot theta / g) H(Xg),
 *    c0 = sqrt(3) e^3 B sin(theta) / (4 pi m c^2), Xg = nu / nu_g,
 *    nu_g = (3/2) nu_B g^2 sin(theta), with the synchrotron functions
 *      F(X) = X int_X^inf K_{5/3},  G(X) = X K_{2/3}(X),
 *      H(X) = X K_{1/3}(X) + int_X^inf K_{1/3}
 *    (Rybicki & Lightman 1979, eqs. 6.31-6.36, for I and Q; H is the
 *    Legg & Westfold circular kernel, whose normalisation is taken so that
 *    a thermal distribution gives the thermal j_V of the thermal module).
 *  - absorption from the Einstein relations in the classical limit for an
 *    isotropic distribution (Rybicki & Lightman eq. 6.50 with p E in place
 *    of E^2, exact for any g): alpha_S = (1 / (2 nu^2 m)) int P_S D dg,
 *    D = -g sqrt(g^2-1) d/dg [N / (g sqrt(g^2-1))]; for the thermal form
 *    D = N / w and alpha_S = j_S / B_nu^RJ exactly (Kirchhoff).
 *  - rotativities: per-electron weights that reproduce the thermal forms
 *    of the thermal module exactly for a Maxwell-Juttner distribution,
 *      rho_V: acosh(g) / (g sqrt(g^2-1))   (mean = K0/K2 for thermal),
 *      rho_Q: (2 g - 1/g) Xg / (1 + Xg)    (mean -> K1/K2 + 6 Theta),
 *    the Xg / (1 + Xg) factor leaving out electrons whose own critical
 *    frequency lies above nu (without it the kappa mean diverges at
 *    kappa = 3); prefactors as in the thermal module.
 *
 * Dimensionless integrals (the eight quantities a surrogate learns; they
 * depend on kappa, w and X = nu / nu_c, nu_c = (3/2) nu_B sin(theta) w^2,
 * only):
 *   I_F = int N F, I_G = int N G, I_H = int N H / g,
 *   A_F = int D F, A_G = int D G, A_H = int D H / g,
 *   R_Q = int N (2g - 1/g) Xg/(1+Xg), R_V = int N acosh(g)/(g sqrt(g^2-1)),
 * with Xg = X w^2 / g^2.
 *
 * Quadrature: u = ln(g - 1) on [-30, 25] with the trapezoid rule, step 0.05
 * (the integrands are analytic in u and negligible at both ends, so the rule
 * converges geometrically).  K_nu and int_x^inf K_nu come from their integral
 * representations int_0^inf exp(-x cosh t) cosh(nu t) [/cosh t] dt, also
 * with the trapezoid rule (even, entire integrands; step 0.05, or 0.25/sqrt(x)
 * where the peak at t = 0 is narrower).
 */
#include <omp.h>
#include <cmath>
#include "oracle_internal.h"

namespace orc {

/* Scaled K_nu(x) e^x and (int_x^inf K_nu) e^x for x > 0. */
static void bessel_reps(double nu, double x, double* k_scaled, double* ki_scaled) {
    /* the integrand is close to exp(-x t^2 / 2) near t = 0: keep h sqrt(x) small */
    const double h = std::fmin(0.05, 0.25 / std::sqrt(x));
    double tmax = std::acosh(1.0 + 80.0 / x) + 1.0;
    int n = (int)(tmax / h) + 1;
    double sk = 0.0, ski = 0.0;
    for (int i = 0; i <= n; ++i) {
        double t = i * h;
        double ch = std::cosh(t);
        double e = std::exp(-x * (ch - 1.0)) * std::cosh(nu * t);
        double wgt = (i == 0) ? 0.5 * h : h;
        sk += wgt * e;
        ski += wgt * e / ch;
    }
    *k_scaled = sk;
    *ki_scaled = ski;
}

double bessel_k(double nu, double x) {
    double k, ki;
    bessel_reps(nu, x, &k, &ki);
    return k * std::exp(-x);
}

double bessel_k_integral(double nu, double x) {
    double k, ki;
    bessel_reps(nu, x, &k, &ki);
    return ki * std::exp(-x);
}

/* F, G, H at X (zero beyond X = 700, where all three are below 1e-300). */
void synchrotron_kernels(double X, double* F, double* G, double* H) {
    if (X > 700.0) {
        *F = *G = *H = 0.0;
        return;
    }
    double k13, ki13, k23, ki23, k53, ki53;
    bessel_reps(1.0 / 3.0, X, &k13, &ki13);
    bessel_reps(2.0 / 3.0, X, &k23, &ki23);
    bessel_reps(5.0 / 3.0, X, &k53, &ki53);
    double ex = std::exp(-X);
    *F = X * ki53 * ex;
    *G = X * k23 * ex;
    *H = (X * k13 + ki13) * ex;
}

void kappa_integrals(int dist, double kappa, double w, double X, double out[8]) {
    const double h = 0.05;
    const int n0 = -600, n1 = 500;   /* u = -30 .. 25 */
    double norm = 0.0, acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int i = n0; i <= n1; ++i) {
        double u = i * h;
        double gm1 = std::exp(u);
        double g = 1.0 + gm1;
        double p = std::sqrt(gm1 * (g + 1.0));
        double f, d;
        if (dist == OR_DIST_KAPPA) {
            double q = 1.0 + gm1 / (kappa * w);
            f = g * p * std::pow(q, -(kappa + 1.0));
            d = f * (kappa + 1.0) / (kappa * w * q);
        } else {
            f = g * p * std::exp(-gm1 / w);
            d = f / w;
        }
        double dg = gm1 * h;
        norm += f * dg;
        double Xg = X * w * w / (g * g);
        double F, G, H;
        synchrotron_kernels(Xg, &F, &G, &H);
        acc[0] += f * F * dg;
        acc[1] += f * G * dg;
        acc[2] += f * H / g * dg;
        acc[3] += d * F * dg;
        acc[4] += d * G * dg;
        acc[5] += d * H / g * dg;
        acc[6] += f * (2.0 * g - 1.0 / g) * Xg / (1.0 + Xg) * dg;
        acc[7] += f * std::acosh(g) / (g * p) * dg;
    }
    for (int k = 0; k < 8; ++k) out[k] = acc[k] / norm;
}

/* Physical coefficients, layout and guards of the thermal module:
 * out = j_I, j_Q, j_V, a_I, a_Q, a_V, r_Q, r_V. */
void kappa_coefficients(int dist, double kappa, double ne, double w, double B, double nu,
                        double cos_thb, double out[8]) {
    for (int k = 0; k < 8; ++k) out[k] = 0.0;
    if (!(ne > 0.0) || !(w > 0.0) || !(B > 0.0) || !(nu > 0.0)) return;
    const double e2 = E_CHARGE * E_CHARGE;
    double c = cos_thb;
    if (c > 1.0) c = 1.0;
    if (c < -1.0) c = -1.0;
    double s = std::sqrt(1.0 - c * c);
    double nuB = E_CHARGE * B / (2.0 * PI * M_ELECTRON * C_LIGHT);
    double nuc = 1.5 * nuB * s * w * w;
    double X = (s > 0.0) ? nu / nuc : INFINITY;
    double I[8];
    kappa_integrals(dist, kappa, w, std::isfinite(X) ? X : 1e300, I);
    out[7] = 2.0 * ne * e2 * nuB * c / (M_ELECTRON * C_LIGHT * nu * nu) * I[7];
    if (s < 1e-10) return;
    double c0 = std::sqrt(3.0) * E_CHARGE * e2 * B * s / (4.0 * PI * M_ELECTRON * C_LIGHT * C_LIGHT);
    double cotv = 4.0 / 3.0 * c / s;
    double jI = ne * c0 * I[0], jQ = ne * c0 * I[1], jV = ne * c0 * cotv * I[2];
    double ab = 1.0 / (2.0 * nu * nu * M_ELECTRON);
    double aI = ne * c0 * I[3] * ab, aQ = ne * c0 * I[4] * ab, aV = ne * c0 * cotv * I[5] * ab;
    double jP = std::hypot(jQ, jV);
    if (jP > jI) {
        jQ *= jI / jP;
        jV *= jI / jP;
    }
    double aP = std::hypot(aQ, aV);
    if (aP > aI) {
        aQ *= aI / aP;
        aV *= aI / aP;
    }
    out[0] = jI;
    out[1] = jQ;
    out[2] = jV;
    out[3] = aI;
    out[4] = aQ;
    out[5] = aV;
    out[6] = ne * e2 * nuB * nuB * s * s / (M_ELECTRON * C_LIGHT * nu * nu * nu) * I[6];
}

}  // namespace orc

extern "C" {
void or_synchrotron_kernels(int64_t n, const double* X, double* out) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) orc::synchrotron_kernels(X[i], &out[3 * i], &out[3 * i + 1], &out[3 * i + 2]);
}
void or_bessel_k(int64_t n, double nu, const double* x, double* k, double* ki) {
    for (int64_t i = 0; i < n; ++i) {
        k[i] = orc::bessel_k(nu, x[i]);
        ki[i] = orc::bessel_k_integral(nu, x[i]);
    }
}
void or_kappa_integrals(int32_t dist, int64_t n, const double* in, double* out, int32_t threads) {
    if (threads <= 0) threads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(threads)
    for (int64_t i = 0; i < n; ++i)
        orc::kappa_integrals(dist, in[3 * i], in[3 * i + 1], in[3 * i + 2], &out[8 * i]);
}
void or_kappa_coefficients(int32_t dist, double kappa, double ne, double w, double B, double nu,
                           double cos_thb, double out[8]) {
    orc::kappa_coefficients(dist, kappa, ne, w, B, nu, cos_thb, out);
}
}
