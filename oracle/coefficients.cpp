/*
 * Thermal synchrotron emission, absorption and Faraday coefficients in the
 * fluid frame.  Test infrastructure only (CPU oracle).
 *
 * Sec. 2.1: the radiative processes are synchrotron emission, synchrotron
 * self-absorption, Faraday rotation and Faraday conversion, for a thermal
 * electron distribution.  The paper cites no fitting formulae; readings:
 *  - emissivities: the thermal fits of Dexter (2016, MNRAS 462, 115, App. A),
 *    in the polarization basis whose second leg lies along the projected
 *    field (so a positive j_Q is emission polarized across the field, as
 *    synchrotron radiation is) and with no U terms;
 *  - absorptivities from Kirchhoff's law, alpha_S = j_S / B_nu(T_e), with
 *    B_nu through expm1 (h nu / k T_e is tiny here);
 *  - rotativities: the thermal-plasma forms with Bessel-function ratios
 *    K0/K2 (rotation) and K1/K2 + 6 Theta_e (conversion), correction factors
 *    set to one;
 *  - guards: no plasma (n_e, Theta_e or B not positive) gives all zeros;
 *    sin(theta_B) < 1e-10 keeps only rho_V; the polarized emissivity is
 *    clamped to j_I.
 */
#include <cmath>
#include "oracle_internal.h"

namespace orc {

/* Asymptotic series of K_nu(x) e^x sqrt(2x/pi) for large x. */
static double kasym(double nu, double x) {
    double mu = 4.0 * nu * nu;
    double term = 1.0, sum = 1.0;
    for (int k = 1; k <= 12; ++k) {
        double odd = 2.0 * k - 1.0;
        term *= (mu - odd * odd) / (k * 8.0 * x);
        sum += term;
    }
    return sum;
}

void bessel_ratios(double x, double* k0k2, double* k1k2) {
    if (x > 700.0) {
        double s0 = kasym(0.0, x), s1 = kasym(1.0, x), s2 = kasym(2.0, x);
        *k0k2 = s0 / s2;
        *k1k2 = s1 / s2;
        return;
    }
    double k0 = std::cyl_bessel_k(0.0, x);
    double k1 = std::cyl_bessel_k(1.0, x);
    double k2 = std::cyl_bessel_k(2.0, x);
    *k0k2 = k0 / k2;
    *k1k2 = k1 / k2;
}

/* out = j_I, j_Q, j_V (erg s^-1 cm^-3 Hz^-1 sr^-1), a_I, a_Q, a_V, r_Q, r_V (cm^-1). */
void thermal_coefficients(double ne, double thetae, double B, double nu, double cos_thb,
                          double out[8]) {
    for (int k = 0; k < 8; ++k) out[k] = 0.0;
    if (!(ne > 0.0) || !(thetae > 0.0) || !(B > 0.0) || !(nu > 0.0)) return;
    const double e2 = E_CHARGE * E_CHARGE;
    double c = cos_thb;
    if (c > 1.0) c = 1.0;
    if (c < -1.0) c = -1.0;
    double s = std::sqrt(1.0 - c * c);
    double nuB = E_CHARGE * B / (2.0 * PI * M_ELECTRON * C_LIGHT);
    double k0k2, k1k2;
    bessel_ratios(1.0 / thetae, &k0k2, &k1k2);

    /* Faraday rotation (kept even along the field) */
    double rV = 2.0 * ne * e2 * nuB * c / (M_ELECTRON * C_LIGHT * nu * nu) * k0k2;
    out[7] = rV;
    if (s < 1e-10) return;

    /* emissivities */
    double nuc = 1.5 * nuB * s * thetae * thetae;
    double x = nu / nuc;
    double xm13 = 1.0 / std::cbrt(x);
    double xm23 = xm13 * xm13;
    double ex = std::exp(-1.8899 * std::cbrt(x));
    double II = 2.5651 * (1.0 + 1.92 * xm13 + 0.9977 * xm23) * ex;
    double IQ = 2.5651 * (1.0 + 0.93193 * xm13 + 0.499873 * xm23) * ex;
    double IV = (1.81348 / x + 3.42319 * xm23 + 0.0292545 / std::sqrt(x) + 2.03773 * xm13) * ex;
    double jI = ne * e2 * nu / (2.0 * std::sqrt(3.0) * C_LIGHT * thetae * thetae) * II;
    double jQ = ne * e2 * nu / (2.0 * std::sqrt(3.0) * C_LIGHT * thetae * thetae) * IQ;
    double jV = 2.0 * ne * e2 * nu * (c / s) / (3.0 * std::sqrt(3.0) * C_LIGHT * thetae * thetae * thetae) * IV;
    double jP = std::hypot(jQ, jV);
    if (jP > jI) {
        jQ *= jI / jP;
        jV *= jI / jP;
    }

    /* Kirchhoff: alpha = j / B_nu(T_e) */
    double Te = thetae * M_ELECTRON * C_LIGHT * C_LIGHT / K_BOLTZ;
    double Bnu = 2.0 * H_PLANCK * nu * nu * nu / (C_LIGHT * C_LIGHT) / std::expm1(H_PLANCK * nu / (K_BOLTZ * Te));
    double aI = 0.0, aQ = 0.0, aV = 0.0;
    if (jI > 0.0 && Bnu > 0.0) {
        aI = jI / Bnu;
        aQ = jQ / Bnu;
        aV = jV / Bnu;
    }

    /* Faraday conversion */
    double rQ = ne * e2 * nuB * nuB * s * s / (M_ELECTRON * C_LIGHT * nu * nu * nu) * (k1k2 + 6.0 * thetae);

    out[0] = jI;
    out[1] = jQ;
    out[2] = jV;
    out[3] = aI;
    out[4] = aQ;
    out[5] = aV;
    out[6] = rQ;
}

}  // namespace orc

extern "C" {
void or_thermal_coefficients(double ne, double thetae, double B, double nu, double cos_thb,
                             double out[8]) {
    orc::thermal_coefficients(ne, thetae, B, nu, cos_thb, out);
}
void or_bessel_ratios(double x, double* k0k2, double* k1k2) { orc::bessel_ratios(x, k0k2, k1k2); }
}
