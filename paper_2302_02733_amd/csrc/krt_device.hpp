// Device math of the polarized Kerr ray tracer (gfx950, FP64).
//
// Everything here follows the method of Sec. 2.1 of Moscibrodzka & Yfantis
// (2023) with the readings stated in krt.h: Kerr-Schild geometry, classical
// RK4 geodesics with the eps step rule, ADAF / snapshot plasma, thermal
// synchrotron coefficients, coherency-matrix transport and the exact
// constant-coefficient Stokes update.  The algebra is arranged for the GPU
// (sparse metric contractions, a closed-form propagator, table-driven Bessel
// ratios); it is mathematically identical to the plain definitions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace krt {

// CODATA 2018, cgs.
constexpr double kC = 2.99792458e10;
constexpr double kG = 6.67430e-8;
constexpr double kH = 6.62607015e-27;
constexpr double kKB = 1.380649e-16;
constexpr double kE = 4.803204712570263e-10;
constexpr double kME = 9.1093837015e-28;
constexpr double kMP = 1.67262192369e-24;
constexpr double kPi = 3.14159265358979323846;

#define KRT_HD __host__ __device__ __forceinline__

// True for finite x (false for inf and NaN).
KRT_HD bool is_finite(double x) { return fabs(x) <= 1.7976931348623157e308; }

// 1/x and 1/sqrt(x) for normal, positive (rcp: non-zero) finite x: the
// hardware estimates (relative error ~5e-8) refined by two Newton steps to
// within an ulp or two, about half the instructions of a correctly rounded
// division or square root.  Callers use them only where the argument is
// bounded away from zero, overflow and subnormals by construction.
KRT_HD double rcp_fast(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
#else
    return 1.0 / x;
#endif
}

KRT_HD double rsqrt_fast(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
    double y = __builtin_amdgcn_rsq(x);
    double h = x * y;
    double e = fma(-h, y, 1.0);
    y = fma(0.5 * y, e, y);
    h = x * y;
    e = fma(-h, y, 1.0);
    return fma(0.5 * y, e, y);
#else
    return 1.0 / sqrt(x);
#endif
}

// sqrt(x) from the reciprocal square root estimate: one Goldschmidt step for
// sqrt and 1/(2 sqrt) together, then one residual correction (within about an
// ulp; the correctly rounded expansion adds a second correction and scaling
// for subnormal arguments: 20 instructions instead of 8).  Arguments at or
// below 1e-290 give 0 (their roots change no term where this is used),
// negative and NaN arguments NaN.
KRT_HD double sqrt_fast(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
    const bool big = x > 1e-290;
    const double xs = big ? x : 1.0;
    const double y = __builtin_amdgcn_rsq(xs);
    double s = xs * y, h = 0.5 * y;
    const double e = fma(-s, h, 0.5);
    s = fma(s, e, s);
    h = fma(h, e, h);
    s = fma(fma(-s, s, xs), h, s);
    return big ? s : (x >= 0.0 ? 0.0 : __builtin_nan(""));
#else
    return sqrt(x);
#endif
}

// sin and cos of a polar angle th in [0, pi]: th is reduced to t in
// [-pi/4, pi/4] around 0, pi/2 or pi (exactly, by Sterbenz's lemma, with the
// low part of pi/2 added after), and sin t, cos t are their Taylor series
// through t^17 and t^16 (truncation below 1e-19 for |t| <= pi/4), in Horner
// form.  A third of the instructions of the general sincos, whose argument
// reduction must handle any angle.
constexpr double kInvFactSin[9] = {1.0, -1.0 / 6.0, 1.0 / 120.0, -1.0 / 5040.0, 1.0 / 362880.0,
                                   -1.0 / 39916800.0, 1.0 / 6227020800.0, -1.0 / 1307674368000.0,
                                   1.0 / 355687428096000.0};
constexpr double kInvFactCos[9] = {1.0, -0.5, 1.0 / 24.0, -1.0 / 720.0, 1.0 / 40320.0,
                                   -1.0 / 3628800.0, 1.0 / 479001600.0, -1.0 / 87178291200.0,
                                   1.0 / 20922789888000.0};

KRT_HD void sincos_polar(double th, double& s, double& c) {
    constexpr double kPio2Hi = 1.5707963267948966;      // nearest double to pi/2
    constexpr double kPio2Lo = 6.123233995736766e-17;   // pi/2 - kPio2Hi
    const int q = th < 0.78539816339744831 ? 0 : (th > 2.3561944901923448 ? 2 : 1);
    const double t = (th - q * kPio2Hi) - q * kPio2Lo;
    const double t2 = t * t;
    double ps = kInvFactSin[8], pc = kInvFactCos[8];
#pragma unroll
    for (int k = 7; k >= 0; --k) {
        ps = fma(ps, t2, kInvFactSin[k]);
        pc = fma(pc, t2, kInvFactCos[k]);
    }
    const double st = ps * t;   // sin t
    // th = q pi/2 + t: (sin, cos) = (st, pc), (pc, -st), (-st, -pc)
    s = q == 0 ? st : (q == 1 ? pc : -st);
    c = q == 0 ? pc : (q == 1 ? -st : -pc);
}

// sin and cos of 2 pi x for any x: reduced to t = 2 pi (x - k/4) in
// [-pi/4, pi/4] (x - k/4 is exact), the quadrant k mod 4 picking the signs.
KRT_HD void sincos_2pi(double x, double& s, double& c) {
    const double k = rint(4.0 * x);
    const double t = 6.283185307179586 * (x - 0.25 * k);
    const double t2 = t * t;
    double ps = kInvFactSin[8], pc = kInvFactCos[8];
#pragma unroll
    for (int j = 7; j >= 0; --j) {
        ps = fma(ps, t2, kInvFactSin[j]);
        pc = fma(pc, t2, kInvFactCos[j]);
    }
    const double st = ps * t;
    const int q = (int)k & 3;
    s = q == 0 ? st : (q == 1 ? pc : (q == 2 ? -st : -pc));
    c = q == 0 ? pc : (q == 1 ? -st : (q == 2 ? -pc : st));
}

// Natural logarithm of a positive normal x: x = m 2^e with m in [sqrt(1/2),
// sqrt(2)), ln m = 2 atanh(u) = 2 (u + u^3/3 + ... + u^21/21), u = (m - 1)/(m + 1)
// (|u| <= 0.172, truncation below 1e-19), plus e ln 2 in two parts.
KRT_HD double log_pos(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
    const int hi = __double2hiint(x);
    int e = ((hi >> 20) & 0x7ff) - 1023;
    int mhi = (hi & 0x000fffff) | 0x3ff00000;
    if (mhi > 0x3ff6a09e) {   // m > sqrt(2): halve it
        mhi -= 0x00100000;
        ++e;
    }
    const double m = __hiloint2double(mhi, __double2loint(x));
#else
    int e;
    double m = 2.0 * frexp(x, &e);
    e -= 1;
    if (m > 1.4142135623730951) {
        m *= 0.5;
        ++e;
    }
#endif
    const double u = (m - 1.0) * rcp_fast(m + 1.0), u2 = u * u;
    double p = 1.0 / 21.0;
#pragma unroll
    for (int k = 19; k >= 1; k -= 2) p = fma(p, u2, 1.0 / k);
    const double lm = 2.0 * u * p;
    return fma((double)e, 1.9082149292705877e-10, lm) + (double)e * 0.6931471803691238;
}

// expm1 for the small arguments of the Planck factor and of the optical
// depth per step: the Taylor series through x^7 for |x| < 1/64 (relative
// truncation below 3e-17), else the library expm1.
KRT_HD double expm1_small(double x) {
    if (fabs(x) < 0.015625)
        return x * (1.0 + x * (0.5 + x * (1.0 / 6.0 + x * (1.0 / 24.0 + x * (1.0 / 120.0 +
                                                                       x * (1.0 / 720.0 + x * (1.0 / 5040.0)))))));
    return expm1(x);
}

// ---------------------------------------------------------------------------
// Kerr-Schild metric at (r, theta): the seven non-zero covariant components,
// their r and theta derivatives, and the six non-zero inverse components.
//   g_tt = f - 1, g_tr = f, g_tp = -a f s^2, g_rr = 1 + f,
//   g_rp = -a s^2 (1 + f), g_hh = Sigma, g_pp = s^2 (Sigma + a^2 s^2 (1 + f)),
//   Sigma = r^2 + a^2 c^2, f = 2 m r / Sigma;
//   g^tt = -(1 + f), g^tr = f, g^rr = Delta / Sigma, g^rp = a / Sigma,
//   g^hh = 1 / Sigma, g^pp = 1 / (Sigma s^2), Delta = r^2 - 2 m r + a^2.
// ---------------------------------------------------------------------------
struct Metric {
    double s, c;                                  // sin, cos theta
    double Sig;
    double tt, tr, tp, rr, rp, hh, pp;            // g_{mu nu}
    double Itt, Itr, Irr, Irp, Ihh, Ipp;          // g^{mu nu}
};

struct MetricD {
    double tt, tr, tp, rr, rp, hh, pp;
};

// Metric at (r, theta) given s = sin(theta), c = cos(theta).
KRT_HD void metric_eval_sc(double a, double m, double r, double s, double c, Metric& g) {
    const double s2 = s * s;
    const double Sig = r * r + a * a * c * c;
    const double iS = rcp_fast(Sig);   // Sigma >= r^2 > 0
    const double f = 2.0 * m * r * iS;
    g.s = s;
    g.c = c;
    g.Sig = Sig;
    g.tt = f - 1.0;
    g.tr = f;
    g.tp = -a * f * s2;
    g.rr = 1.0 + f;
    g.rp = -a * s2 * (1.0 + f);
    g.hh = Sig;
    g.pp = s2 * (Sig + a * a * s2 * (1.0 + f));
    g.Itt = -(1.0 + f);
    g.Itr = f;
    g.Irr = (r * r - 2.0 * m * r + a * a) * iS;
    g.Irp = a * iS;
    g.Ihh = iS;
    g.Ipp = iS * rcp_fast(s2);          // sin^2 theta >= 1e-24 on any stored point
}

KRT_HD void metric_eval(double a, double m, double r, double th, Metric& g) {
    double s, c;
    sincos(th, &s, &c);
    metric_eval_sc(a, m, r, s, c, g);
}

// Metric plus its r- and theta-derivatives, given sin and cos of theta.
KRT_HD void metric_eval_d_sc(double a, double m, double r, double sn, double cs, Metric& g,
                             MetricD& dr, MetricD& dh) {
    metric_eval_sc(a, m, r, sn, cs, g);
    const double s = g.s, c = g.c, s2 = s * s, sc = s * c;
    const double Sig = g.Sig, iS = rcp_fast(Sig);
    const double f = g.tr;
    const double Sig_h = -2.0 * a * a * sc;
    const double f_r = 2.0 * m * (a * a * c * c - r * r) * iS * iS;
    const double f_h = -f * Sig_h * iS;
    const double s2_h = 2.0 * sc;
    const double opf = 1.0 + f;
    dr.tt = f_r;
    dr.tr = f_r;
    dr.tp = -a * s2 * f_r;
    dr.rr = f_r;
    dr.rp = -a * s2 * f_r;
    dr.hh = 2.0 * r;
    dr.pp = s2 * (2.0 * r + a * a * s2 * f_r);
    dh.tt = f_h;
    dh.tr = f_h;
    dh.tp = -a * (f_h * s2 + f * s2_h);
    dh.rr = f_h;
    dh.rp = -a * (s2_h * opf + s2 * f_h);
    dh.hh = Sig_h;
    dh.pp = s2_h * (Sig + a * a * s2 * opf) + s2 * (Sig_h + a * a * (s2_h * opf + s2 * f_h));
}

KRT_HD void metric_eval_d(double a, double m, double r, double th, Metric& g, MetricD& dr,
                          MetricD& dh) {
    double s, c;
    sincos(th, &s, &c);
    metric_eval_d_sc(a, m, r, s, c, g, dr, dh);
}

// Lower a vector: v_mu = g_{mu nu} v^nu.
KRT_HD void lower(const Metric& g, const double v[4], double o[4]) {
    o[0] = g.tt * v[0] + g.tr * v[1] + g.tp * v[3];
    o[1] = g.tr * v[0] + g.rr * v[1] + g.rp * v[3];
    o[2] = g.hh * v[2];
    o[3] = g.tp * v[0] + g.rp * v[1] + g.pp * v[3];
}

// Raise a covector: v^mu = g^{mu nu} v_nu.
KRT_HD void raise(const Metric& g, const double v[4], double o[4]) {
    o[0] = g.Itt * v[0] + g.Itr * v[1];
    o[1] = g.Itr * v[0] + g.Irr * v[1] + g.Irp * v[3];
    o[2] = g.Ihh * v[2];
    o[3] = g.Irp * v[1] + g.Ipp * v[3];
}

KRT_HD double dot(const Metric& g, const double x[4], const double y[4]) {
    double yl[4];
    lower(g, y, yl);
    return x[0] * yl[0] + x[1] * yl[1] + x[2] * yl[2] + x[3] * yl[3];
}

// D . K for a derivative D of the metric (a covector).
KRT_HD void dmetric_times(const MetricD& d, const double K[4], double o[4]) {
    o[0] = d.tt * K[0] + d.tr * K[1] + d.tp * K[3];
    o[1] = d.tr * K[0] + d.rr * K[1] + d.rp * K[3];
    o[2] = d.hh * K[2];
    o[3] = d.tp * K[0] + d.rp * K[1] + d.pp * K[3];
}

// Geodesic acceleration dK^mu/dlam = -Gamma^mu_ab K^a K^b, written as
// -g^{mu nu} [K^r (D_r K)_nu + K^h (D_h K)_nu - 1/2 delta_nu^{r,h} K.D K]
// (only r and theta derivatives are non-zero), with the Kerr-Schild
// derivatives factored: d_r g_tt = d_r g_tr = d_r g_rr = f_r and
// d_r g_tp = d_r g_rp = -a s^2 f_r, so with P = K^t + K^r - a s^2 K^p,
//   (D_r K)_t = (D_r K)_r = f_r P,  (D_r K)_h = 2 r K^h,
//   (D_r K)_p = -a s^2 f_r P + 2 r s^2 K^p,  K.D_r K = f_r P^2 + 2 r (K^h^2 + s^2 K^p^2);
// d_h g_tt = d_h g_tr = d_h g_rr = f_h and d_h g_rp = d_h g_tp - a (s^2)_h, so
// (D_h K)_r = (D_h K)_t - a (s^2)_h K^p.
KRT_HD void geodesic_acc_sc(double a, double m, double r, double sn, double cs, const double K[4],
                            double acc[4]) {
    const double s2 = sn * sn, c2 = cs * cs, sc = sn * cs, a2 = a * a;
    const double Sig = r * r + a2 * c2;
    const double iS = rcp_fast(Sig);
    const double f = 2.0 * m * r * iS;
    const double opf = 1.0 + f;
    // derivatives
    const double f_r = 2.0 * m * (a2 * c2 - r * r) * iS * iS;
    const double Sig_h = -2.0 * a2 * sc;
    const double f_h = -f * Sig_h * iS;
    const double s2_h = 2.0 * sc;
    const double gtp_h = -a * (f_h * s2 + f * s2_h);
    const double grp_h = gtp_h - a * s2_h;
    const double gpp_h = s2_h * (Sig + a2 * s2 * opf) + s2 * (Sig_h + a2 * (s2_h * opf + s2 * f_h));
    const double Kt = K[0], Kr = K[1], Kh = K[2], Kp = K[3];
    const double Ktr = Kt + Kr;
    // D_r K and D_h K
    const double as2 = a * s2;
    const double P = Ktr - as2 * Kp;
    const double vr0 = f_r * P;
    const double vr2 = 2.0 * r * Kh;
    const double vr3 = 2.0 * r * s2 * Kp - as2 * vr0;
    const double vh0 = f_h * Ktr + gtp_h * Kp;
    const double vh1 = vh0 - a * s2_h * Kp;
    const double vh2 = Sig_h * Kh;
    const double vh3 = gtp_h * Kt + grp_h * Kr + gpp_h * Kp;
    const double Qr = vr0 * P + 2.0 * r * (Kh * Kh + s2 * Kp * Kp);
    const double Qh = Kt * vh0 + Kr * vh1 + Kh * vh2 + Kp * vh3;
    const double w0 = Kr * vr0 + Kh * vh0;
    const double w1 = Kr * vr0 + Kh * vh1 - 0.5 * Qr;
    const double w2 = Kr * vr2 + Kh * vh2 - 0.5 * Qh;
    const double w3 = Kr * vr3 + Kh * vh3;
    // -g^{mu nu} w_nu: g^tt = -(1 + f), g^tr = f, g^rr = Delta / Sigma,
    // g^rp = a / Sigma, g^hh = 1 / Sigma, g^pp = 1 / (Sigma s^2)
    acc[0] = opf * w0 - f * w1;
    acc[1] = -(f * w0 + ((r * r - 2.0 * m * r + a2) * w1 + a * w3) * iS);
    acc[2] = -w2 * iS;
    acc[3] = -(a * w1 + w3 * rcp_fast(s2)) * iS;
}

KRT_HD void geodesic_acc(double a, double m, double r, double th, const double K[4],
                         double acc[4]) {
    double s, c;
    sincos(th, &s, &c);
    geodesic_acc_sc(a, m, r, s, c, K, acc);
}

// Connection along the ray A^mu_b = Gamma^mu_ab K^a =
// 1/2 g^{mu nu} T_{nu b},  T_{nu b} = M_{nu b} + delta_b^r (D_r K)_nu + delta_b^h (D_h K)_nu
//                                    - delta_nu^r (D_r K)_b - delta_nu^h (D_h K)_b,
// M = K^r D_r g + K^h D_h g.  Written out entry by entry: the Kerr-Schild
// metric and its derivatives have no (t,h), (r,h) or (h,p) components, so
// T_rr = M_rr and T_hh = M_hh, and each sum runs over the non-zero terms only
// (a product with a structural zero is not free in IEEE arithmetic).
// A is returned row-major, A[mu][b].
KRT_HD void connection(const Metric& g, const MetricD& dr, const MetricD& dh, const double K[4],
                       double A[16]) {
    double vr[4], vh[4];
    dmetric_times(dr, K, vr);
    dmetric_times(dh, K, vh);
    const double kr = K[1], kh = K[2];
    const double Mtt = kr * dr.tt + kh * dh.tt, Mtr = kr * dr.tr + kh * dh.tr;
    const double Mtp = kr * dr.tp + kh * dh.tp, Mrr = kr * dr.rr + kh * dh.rr;
    const double Mrp = kr * dr.rp + kh * dh.rp, Mhh = kr * dr.hh + kh * dh.hh;
    const double Mpp = kr * dr.pp + kh * dh.pp;
    // T rows t, r, h, p (columns t, r, h, p)
    const double Ttt = Mtt, Ttr = Mtr + vr[0], Tth = vh[0], Ttp = Mtp;
    const double Trt = Mtr - vr[0], Trr = Mrr, Trh = vh[1] - vr[2], Trp = Mrp - vr[3];
    const double Tht = -vh[0], Thr = vr[2] - vh[1], Thh = Mhh, Thp = -vh[3];
    const double Tpt = Mtp, Tpr = Mrp + vr[3], Tph = vh[3], Tpp = Mpp;
    const double htt = 0.5 * g.Itt, htr = 0.5 * g.Itr, hrr = 0.5 * g.Irr, hrp = 0.5 * g.Irp;
    const double hhh = 0.5 * g.Ihh, hpp = 0.5 * g.Ipp;
    A[0] = htt * Ttt + htr * Trt;
    A[1] = htt * Ttr + htr * Trr;
    A[2] = htt * Tth + htr * Trh;
    A[3] = htt * Ttp + htr * Trp;
    A[4] = htr * Ttt + hrr * Trt + hrp * Tpt;
    A[5] = htr * Ttr + hrr * Trr + hrp * Tpr;
    A[6] = htr * Tth + hrr * Trh + hrp * Tph;
    A[7] = htr * Ttp + hrr * Trp + hrp * Tpp;
    A[8] = hhh * Tht;
    A[9] = hhh * Thr;
    A[10] = hhh * Thh;
    A[11] = hhh * Thp;
    A[12] = hrp * Trt + hpp * Tpt;
    A[13] = hrp * Trr + hpp * Tpr;
    A[14] = hrp * Trh + hpp * Tph;
    A[15] = hrp * Trp + hpp * Tpp;
}

// ---------------------------------------------------------------------------
// Camera: SplitMix64 jitter (Steele, Lea & Flood 2014 output function),
// static-observer tetrad by Gram-Schmidt of (d_t, d_r, d_theta, d_phi), photon
// launch K = e0 + n and the pixel's screen legs.
// ---------------------------------------------------------------------------
KRT_HD uint64_t splitmix64_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

KRT_HD double pixel_jitter(uint64_t seed, uint64_t counter) {
    const uint64_t z = splitmix64_mix(seed + counter * 0x9E3779B97F4A7C15ULL);
    return (double)(z >> 11) * 0x1.0p-53 - 0.5;
}

struct CameraDesc {
    double a, m, r_cam, th, ph, fov_x, fov_y, freq;
    int nx, ny, jitter;
    uint64_t seed;
};

KRT_HD void pixel_position(const CameraDesc& cd, int i, int j, double& alpha, double& beta) {
    double dx = 0.0, dy = 0.0;
    if (cd.jitter) {
        const uint64_t k = 2ULL * ((uint64_t)j * (uint64_t)cd.nx + (uint64_t)i);
        dx = pixel_jitter(cd.seed, k + 1ULL);
        dy = pixel_jitter(cd.seed, k + 2ULL);
    }
    alpha = cd.fov_x * ((i + 0.5 + dx) / cd.nx - 0.5);
    beta = cd.fov_y * ((j + 0.5 + dy) / cd.ny - 0.5);
}

// Static observer's orthonormal tetrad e[0..3] (contravariant) at the camera.
KRT_HD void camera_tetrad(const CameraDesc& cd, const Metric& g, double e[4][4]) {
    for (int k = 0; k < 4; ++k)
        for (int mu = 0; mu < 4; ++mu) e[k][mu] = (k == mu) ? 1.0 : 0.0;
    e[0][0] = 1.0 / sqrt(-g.tt);
    for (int k = 1; k < 4; ++k) {
        double v[4] = {e[k][0], e[k][1], e[k][2], e[k][3]};
        const double p0 = dot(g, v, e[0]);
        for (int mu = 0; mu < 4; ++mu) v[mu] += p0 * e[0][mu];
        for (int l = 1; l < k; ++l) {
            const double pl = dot(g, v, e[l]);
            for (int mu = 0; mu < 4; ++mu) v[mu] -= pl * e[l][mu];
        }
        const double inv = 1.0 / sqrt(dot(g, v, v));
        for (int mu = 0; mu < 4; ++mu) e[k][mu] = v[mu] * inv;
    }
}

// Direction of travel of the arriving photon in the camera frame
// (components on e_r, e_theta, e_phi).
KRT_HD void arrival_direction(const CameraDesc& cd, double alpha, double beta, double n[3]) {
    const double ra = alpha / cd.r_cam, rb = beta / cd.r_cam;
    const double inv = 1.0 / sqrt(1.0 + ra * ra + rb * rb);
    n[0] = inv;
    n[1] = rb * inv;
    n[2] = -ra * inv;
}

KRT_HD void camera_launch(const CameraDesc& cd, double alpha, double beta, double X[4],
                          double K[4]) {
    Metric g;
    metric_eval(cd.a, cd.m, cd.r_cam, cd.th, g);
    double e[4][4];
    camera_tetrad(cd, g, e);
    double n[3];
    arrival_direction(cd, alpha, beta, n);
    X[0] = 0.0;
    X[1] = cd.r_cam;
    X[2] = cd.th;
    X[3] = cd.ph;
    for (int mu = 0; mu < 4; ++mu) K[mu] = e[0][mu] + n[0] * e[1][mu] + n[1] * e[2][mu] + n[2] * e[3][mu];
}

// Screen legs of a pixel: e_x = e_phi, e_y = -e_theta made transverse to the
// pixel's arrival direction: x' = normalised(x - (x.n) n), y' = n cross x'.
KRT_HD void screen_legs(const CameraDesc& cd, const Metric& g, double alpha, double beta,
                        double ex[4], double ey[4]) {
    double e[4][4];
    camera_tetrad(cd, g, e);
    double n[3];
    arrival_direction(cd, alpha, beta, n);
    double x[3] = {-n[2] * n[0], -n[2] * n[1], 1.0 - n[2] * n[2]};
    const double inv = 1.0 / sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    x[0] *= inv;
    x[1] *= inv;
    x[2] *= inv;
    const double y[3] = {n[1] * x[2] - n[2] * x[1], n[2] * x[0] - n[0] * x[2],
                         n[0] * x[1] - n[1] * x[0]};
    for (int mu = 0; mu < 4; ++mu) {
        ex[mu] = x[0] * e[1][mu] + x[1] * e[2][mu] + x[2] * e[3][mu];
        ey[mu] = y[0] * e[1][mu] + y[1] * e[2][mu] + y[2] * e[3][mu];
    }
}

// ---------------------------------------------------------------------------
// Plasma.
// ---------------------------------------------------------------------------
struct Plasma {
    double ne, thetae, B;
    double u[4], b[4];
    double bb;   // b.b (the model forms it; the transfer and the tetrad reuse it)
};

struct AdafDesc {
    double n0, T0, beta, h, risco;
    double ibeta, i2h2;   // 1 / beta and 1 / (2 h^2), formed on the host
};

// Analytic ADAF-like flow.  Returns false where no timelike flow exists.
KRT_HD bool adaf_plasma(const AdafDesc& ad, double a, double m, double r, const Metric& g,
                        Plasma& p) {
    const double c = g.c;
    // r^(1/2), 1/r and r^(-3/2) from one reciprocal square root (r > 1)
    const double irs = rsqrt_fast(r);
    const double sr = r * irs, ir = irs * irs;
    p.ne = ad.n0 * (ir * irs) * exp(-c * c * ad.i2h2);
    p.thetae = (kKB / (kME * kC * kC)) * ad.T0 * ir;
    p.B = sqrt_fast((8.0 * kPi * kMP * kC * kC / 6.0) * p.ne * ir * ad.ibeta);
    double Om = 0.0, norm = 1.0;
    const bool kepler = (m != 0.0) && (r >= ad.risco);
    if (kepler) {
        Om = rcp_fast(r * sr + a);
        norm = g.tt + 2.0 * g.tp * Om + g.pp * Om * Om;
    }
    if (!kepler || !(norm < 0.0)) {
        Om = -g.tp / g.pp;
        norm = g.tt + 2.0 * g.tp * Om + g.pp * Om * Om;
    }
    if (!(norm < 0.0)) return false;
    const double ut = rsqrt_fast(-norm);
    p.u[0] = ut;
    p.u[1] = 0.0;
    p.u[2] = 0.0;
    p.u[3] = Om * ut;
    // toroidal field b = B (d_phi + u_phi u) / sqrt(g_pp + u_phi^2)
    const double uph = g.tp * ut + g.pp * p.u[3];
    const double sc = p.B * rsqrt_fast(g.pp + uph * uph);
    p.b[0] = sc * uph * p.u[0];
    p.b[1] = 0.0;
    p.b[2] = 0.0;
    p.b[3] = sc * (1.0 + uph * p.u[3]);
    p.bb = p.B * p.B;   // b.b = B^2 by construction
    return true;
}

// Gridded snapshot on a modified Kerr-Schild grid: x1 = ln r,
// theta = pi x2 + (1 - h)/2 sin(2 pi x2), x3 = phi; cell-centred primitives
// (rho, u, U1, U2, U3, B1, B2, B3), layout [n1][n2][n3][8].
struct SnapDesc {
    const double* prims;       // FP64 primitives, or null when prims_f is set
    const float* prims_f;      // FP32 primitives (same layout)
    int n1, n2, n3;
    double x1s, dx1, x2s, dx2, x3s, dx3;
    double idx1, idx2, idx3;   // 1 / dx, formed on the host
    double in3;                // 1 / n3, formed on the host
    double h, gam;
    double rho_unit, B_unit;   // M_unit / L^3 and c sqrt(4 pi rho_unit)
    double Rhigh, Rlow, sigma_cut, rmax;
    // x2 at theta = k pi / kX2Tab, k = 0..kX2Tab (the MKS inversion's start
    // values; null: start from theta / pi)
    const double* x2tab;
};

constexpr int kX2Tab = 1024;

// Start value of the MKS inversion x2(theta): linear interpolation in the
// table (error below 2e-5 for hslope 0.3, which two Newton steps take below
// the resolution of x2), or theta / pi without a table.
KRT_HD double x2_start(const double* tab, double th) {
    if (!tab) return th * (1.0 / kPi);
    const double u = th * (kX2Tab / kPi);
    double fi = floor(u);
    fi = fi >= 0.0 ? (fi > kX2Tab - 1 ? kX2Tab - 1 : fi) : 0.0;   // (NaN: 0)
    const int i = (int)fi;
    const double a = tab[i], b = tab[i + 1];
    return fma(u - fi, b - a, a);
}

// Trilinear interpolation at grid coordinates; clamped to the end cells in
// x1 and x2, periodic in x3.
KRT_HD void snapshot_interp(const SnapDesc& s, double x1, double x2, double x3, double P[8]) {
    int i0[3], i1[3];
    double d[3];
    const double X0 = (x1 - s.x1s) * s.idx1 - 0.5, X1 = (x2 - s.x2s) * s.idx2 - 0.5;
    const double Xv[2] = {X0, X1};
    const int nn[2] = {s.n1, s.n2};
    for (int k = 0; k < 2; ++k) {
        const double f = floor(Xv[k]);
        int i = (int)f;
        double t = Xv[k] - f;
        if (i < 0) { i = 0; t = 0.0; }
        if (i > nn[k] - 2) { i = nn[k] - 2; t = 1.0; }
        i0[k] = i;
        i1[k] = i + 1;
        d[k] = t;
    }
    {
        const double X2 = (x3 - s.x3s) * s.idx3 - 0.5;
        const double f = floor(X2);
        // the cell index f mod n3 in integer-valued FP64 (exact; the
        // quotient's rounding is corrected by one period) instead of integer
        // remainders
        const double n = (double)s.n3;
        double fi = f - n * floor(f * s.in3);
        fi = fi < 0.0 ? fi + n : (fi >= n ? fi - n : fi);
        const int i = (int)fi;
        i0[2] = i;
        i1[2] = i + 1 == s.n3 ? 0 : i + 1;
        d[2] = X2 - f;
    }
    for (int q = 0; q < 8; ++q) P[q] = 0.0;
    for (int c = 0; c < 8; ++c) {
        const int ia = (c & 4) ? i1[0] : i0[0];
        const int ib = (c & 2) ? i1[1] : i0[1];
        const int ic = (c & 1) ? i1[2] : i0[2];
        const double w = ((c & 4) ? d[0] : 1.0 - d[0]) * ((c & 2) ? d[1] : 1.0 - d[1]) *
                         ((c & 1) ? d[2] : 1.0 - d[2]);
        const size_t off = 8 * (((size_t)ia * s.n2 + ib) * s.n3 + ic);
        if (s.prims_f) {
            const float4* cell = reinterpret_cast<const float4*>(s.prims_f + off);
            const float4 v0 = cell[0], v1 = cell[1];
            P[0] += w * v0.x; P[1] += w * v0.y; P[2] += w * v0.z; P[3] += w * v0.w;
            P[4] += w * v1.x; P[5] += w * v1.y; P[6] += w * v1.z; P[7] += w * v1.w;
        } else {
            const double2* cell = reinterpret_cast<const double2*>(s.prims + off);
            const double2 v0 = cell[0], v1 = cell[1], v2 = cell[2], v3 = cell[3];
            P[0] += w * v0.x; P[1] += w * v0.y; P[2] += w * v1.x; P[3] += w * v1.y;
            P[4] += w * v2.x; P[5] += w * v2.y; P[6] += w * v3.x; P[7] += w * v3.y;
        }
    }
}

// Plasma from the snapshot.  The grid velocity and field components are
// mapped to Kerr-Schild with the diagonal Jacobian (1, r, dtheta/dx2, 1);
// then u^t = gamma / lapse, u^i = U^i - gamma lapse g^{ti} with
// gamma = sqrt(1 + g_ij U^i U^j) and lapse = 1/sqrt(-g^tt); b^t = B^i u_i,
// b^i = (B^i + b^t u^i) / u^t; T_i/T_e = (R_high beta^2 + R_low)/(1 + beta^2)
// with beta = (gamma_ad - 1) u / (b.b/2); no emission (n_e = 0) where
// b.b/rho > sigma_cut or r > r_emit_max.
// Returns 1, or 2 when the gathered primitives are not finite (the caller
// poisons the ray: its pixel is written as NONFINITE).
KRT_HD int snapshot_plasma(const SnapDesc& s, double a, double m, double r, double th, double ph,
                           const Metric& g, Plasma& p) {
    const double x1 = log_pos(r);
    double x2 = x2_start(s.x2tab, th);
    const double hh = 0.5 * (1.0 - s.h);
    // Newton from the tabulated start: quadratic convergence, at most 8
    // steps, stopping once a step no longer moves x2 beyond round-off
    double cs = 1.0;
    for (int it = 0; it < 8; ++it) {
        double sn;
        sincos_2pi(x2, sn, cs);
        const double dx = (kPi * x2 + hh * sn - th) * rcp_fast(kPi * (1.0 + (1.0 - s.h) * cs));
        x2 -= dx;
        if (fabs(dx) < 1e-15) break;
    }
    double P[8];
    snapshot_interp(s, x1, x2, ph, P);
    if (!is_finite(P[0] + P[1] + P[2] + P[3] + P[4] + P[5] + P[6] + P[7])) return 2;
    const double rho = P[0], uu = P[1];
    // dtheta/dx2 with the last Newton step's cosine (after the converged
    // step x2 has moved by less than 1e-15)
    const double J2 = kPi * (1.0 + (1.0 - s.h) * cs);
    const double U[4] = {0.0, P[2] * r, P[3] * J2, P[4]};
    const double Bv[4] = {0.0, P[5] * r, P[6] * J2, P[7]};
    // g_ij U^i U^j (spatial part)
    const double q = g.rr * U[1] * U[1] + 2.0 * g.rp * U[1] * U[3] + g.hh * U[2] * U[2] + g.pp * U[3] * U[3];
    const double gamma = sqrt_fast(1.0 + q);
    const double lapse = rsqrt_fast(-g.Itt);
    p.u[0] = gamma * (-g.Itt * lapse);   // gamma / lapse
    p.u[1] = U[1] - gamma * lapse * g.Itr;
    p.u[2] = U[2];
    p.u[3] = U[3];
    double ul[4];
    lower(g, p.u, ul);
    const double bt = Bv[1] * ul[1] + Bv[2] * ul[2] + Bv[3] * ul[3];
    const double iut = rcp_fast(p.u[0]);
    p.b[0] = bt;
    p.b[1] = (Bv[1] + bt * p.u[1]) * iut;
    p.b[2] = (Bv[2] + bt * p.u[2]) * iut;
    p.b[3] = (Bv[3] + bt * p.u[3]) * iut;
    const double bsq = dot(g, p.b, p.b);
    p.bb = bsq;
    p.B = sqrt_fast(bsq > 0.0 ? bsq : 0.0) * s.B_unit;
    p.ne = rho * s.rho_unit * (1.0 / (kMP + kME));
    double thetae = 0.0;
    if (rho > 0.0 && uu > 0.0) {
        // 1/beta = (b.b/2) / ((gamma_ad - 1) u); T_i/T_e = (R_high + R_low / beta^2) / (1 + 1/beta^2)
        const double ib = 0.5 * bsq * rcp_fast((s.gam - 1.0) * uu);
        const double ib2 = ib * ib;
        const double iden = rcp_fast(1.0 + ib2);
        const double trat = (s.Rhigh + s.Rlow * ib2) * iden;
        thetae = (kMP / kME) * (s.gam - 1.0) * uu * rcp_fast(rho * (1.0 + trat));
    }
    p.thetae = thetae;
    if (!(rho > 0.0) || bsq > s.sigma_cut * rho || r > s.rmax) p.ne = 0.0;
    (void)a;
    (void)m;
    return 1;
}

// ---------------------------------------------------------------------------
// Bessel-function ratios K0/K2 and K1/K2 of x = 1/Theta_e.
// Table: piecewise polynomials of degree kBesDeg in x itself, on panels
// that split every binade [2^e, 2^(e+1)) of [2^kBesE0, 2^kBesE1) into
// kBesSub equal parts, built at context creation from the trapezoid rule on
// K_nu(x) e^x = int_0^inf exp(-x (cosh s - 1)) cosh(nu s) ds as Chebyshev
// interpolants and stored as monomial coefficients in the panel variable z
// (evaluated by Horner's rule, one FMA per degree; the Chebyshev coefficients
// decay fast enough on these panels that both forms round alike).  A panel and
// its Chebyshev variable come from the exponent and mantissa bits of x (no
// logarithm); the ratios are analytic in x away from x = 0, which lies 8 panel
// half-widths or more from every panel, so degree 12 reaches round-off.
// Outside [1e-8, 700]: leading small-x forms, the asymptotic series above.
// ---------------------------------------------------------------------------
constexpr int kBesE0 = -27;                      // 2^-27 < 1e-8
constexpr int kBesE1 = 10;                       // 2^10 > 700
constexpr int kBesSub = 4;                       // panels per binade
constexpr int kBesPanels = (kBesE1 - kBesE0) * kBesSub;
constexpr int kBesDeg = 12;
constexpr int kBesCoef = kBesDeg + 1;

// Panel of x in [2^kBesE0, 2^kBesE1) and the Chebyshev variable z in [-1, 1]
// there: x = m 2^e with m in [1, 2); sub-panel k = floor(4 (m - 1)) (the top two
// mantissa bits); z = 8 (m - 1) - (2 k + 1).
KRT_HD int bessel_panel(double x, double& z) {
#if defined(__HIP_DEVICE_COMPILE__)
    const int hi = __double2hiint(x);
    const int e = ((hi >> 20) & 0x7ff) - 1023;
    const int k = (hi >> 18) & (kBesSub - 1);
    const double m = __hiloint2double((hi & 0x000fffff) | 0x3ff00000, __double2loint(x));
#else
    int e;
    const double m = 2.0 * frexp(x, &e);
    e -= 1;
    const int k = (int)((m - 1.0) * kBesSub);
#endif
    z = 8.0 * m - (double)(9 + 2 * k);
    int p = (e - kBesE0) * kBesSub + k;
    return p < 0 ? 0 : (p >= kBesPanels ? kBesPanels - 1 : p);
}

// x at Chebyshev variable z of panel p (table construction).
KRT_HD double bessel_panel_x(int p, double z) {
    const int e = kBesE0 + p / kBesSub, k = p % kBesSub;
    return ldexp(1.0 + (2 * k + 1 + z) * 0.125, e);
}

// Asymptotic series of sqrt(2x/pi) e^x K_nu(x) for large x.
KRT_HD double bessel_k_asym_series(double nu, double x) {
    const double mu = 4.0 * nu * nu;
    double term = 1.0, sum = 1.0;
    for (int k = 1; k <= 12; ++k) {
        const double o = 2.0 * k - 1.0;
        term *= (mu - o * o) / (8.0 * k * x);
        sum += term;
    }
    return sum;
}

KRT_HD void bessel_ratios(const double* __restrict__ table, double x,
                                              double& k0k2, double& k1k2) {
    if (x > 700.0) {
        const double s0 = bessel_k_asym_series(0.0, x), s1 = bessel_k_asym_series(1.0, x);
        const double s2 = bessel_k_asym_series(2.0, x);
        k0k2 = s0 / s2;
        k1k2 = s1 / s2;
        return;
    }
    if (x < 1e-8) {
        k0k2 = 0.5 * x * x * (-log(0.5 * x) - 0.57721566490153286);
        k1k2 = 0.5 * x;
        return;
    }
    double z;
    const int p = bessel_panel(x, z);
    const double* c0 = table + (size_t)p * 2 * kBesCoef;
    const double* c1 = c0 + kBesCoef;
    double b = c0[kBesDeg], d = c1[kBesDeg];
    for (int k = kBesDeg - 1; k >= 0; --k) {
        b = fma(b, z, c0[k]);
        d = fma(d, z, c1[k]);
    }
    k0k2 = b;
    k1k2 = d;
}

// ---------------------------------------------------------------------------
// Thermal synchrotron coefficients in the fluid frame (cgs): emissivities of
// Dexter (2016, App. A) in the basis whose second leg is along the projected
// field, Kirchhoff absorptivities, thermal rotativities.  Writes
// (j_I, j_Q, j_V, a_I, a_Q, a_V, r_Q, r_V) and returns the source function
// B_nu / nu^3 = (2 h / c^2) / expm1(h nu / k T_e) where a_I > 0 (else 0).
// Constant factors are folded and divisions shared: 1/Theta_e, 1/nu,
// nu_c / nu, x^-1/3 and 1/B_nu are the only reciprocals.
// ---------------------------------------------------------------------------
constexpr double kNuBPerB = kE / (2.0 * kPi * kME * kC);          // nu_B / B
constexpr double kRhoVFac = 2.0 * kE * kE / (kME * kC);          // r_V prefactor
constexpr double kJIFac = kE * kE / (2.0 * 1.7320508075688772 * kC);
constexpr double kHnuOverTheta = kH / (kME * kC * kC);           // h nu / (k T_e) = this nu / Theta_e
constexpr double kSrcFac = 2.0 * kH / (kC * kC);

KRT_HD double thermal_coefficients(const double* __restrict__ btab, double ne, double thetae,
                                   double B, double nu, double cth, double out[8]) {
    for (int k = 0; k < 8; ++k) out[k] = 0.0;
    if (!(ne > 0.0) || !(thetae > 0.0) || !(B > 0.0) || !(nu > 0.0)) return 0.0;
    cth = cth > 1.0 ? 1.0 : (cth < -1.0 ? -1.0 : cth);
    // sin(theta_B) and its reciprocal from one reciprocal square root
    const double s2th = 1.0 - cth * cth;
    const double isth = s2th > 1e-200 ? rsqrt_fast(s2th) : 0.0;
    const double sth = s2th * isth;
    const double nuB = kNuBPerB * B;
    const double iTh = rcp_fast(thetae);
    double k0k2, k1k2;
    bessel_ratios(btab, iTh, k0k2, k1k2);
    const double inu = rcp_fast(nu);
    const double inu2 = inu * inu;
    out[7] = kRhoVFac * ne * nuB * cth * inu2 * k0k2;
    if (sth < 1e-10) return 0.0;
    out[6] = 0.5 * kRhoVFac * ne * nuB * nuB * sth * sth * inu2 * inu * (k1k2 + 6.0 * thetae);

    const double nuc = 1.5 * nuB * sth * thetae * thetae;
    // x^(-1/3) from the reciprocal cube root, x^(1/3) = x x^(-2/3)
    const double xx = nu * rcp_fast(nuc);
#if defined(__HIP_DEVICE_COMPILE__)
    const double xm13 = rcbrt(xx);
#else
    const double xm13 = 1.0 / cbrt(xx);
#endif
    const double xm23 = xm13 * xm13;
    const double x13 = xx * xm23;
    const double ex = exp(-1.8899 * x13);
    const double II = 2.5651 * (1.0 + 1.92 * xm13 + 0.9977 * xm23) * ex;
    const double IQ = 2.5651 * (1.0 + 0.93193 * xm13 + 0.499873 * xm23) * ex;
    // x^-1 = xm13^3, x^-1/2 = xm13^(3/2)
    const double IV = (1.81348 * xm23 * xm13 + 3.42319 * xm23 + 0.0292545 * xm13 * sqrt_fast(xm13) +
                       2.03773 * xm13) * ex;
    const double pre = kJIFac * ne * nu * iTh * iTh;
    double jI = pre * II;
    double jQ = pre * IQ;
    // j_V = 2 ne e^2 nu cot(theta_B) IV / (3 sqrt3 c Theta^3) = pre (4/3) cot(theta_B) IV / Theta
    double jV = pre * (4.0 / 3.0) * (cth * isth) * iTh * IV;
    // clamp |j_P| <= j_I, compared in squares where they stay normal numbers
    // (j_I in 1e-140..1e140, |j_Q|, |j_V| below 1e10 j_I); hypot elsewhere
    const bool sq = jI > 1e-140 && jI < 1e140;
    if (sq ? (jQ * jQ + jV * jV > jI * jI) : (hypot(jQ, jV) > jI)) {
        const double sc = jI / hypot(jQ, jV);
        jQ *= sc;
        jV *= sc;
    }
    out[0] = jI;
    out[1] = jQ;
    out[2] = jV;
    const double em1 = expm1_small(kHnuOverTheta * nu * iTh);
    const double seq = kSrcFac * rcp_fast(em1);
    const double Bnu = seq * nu * nu * nu;
    if (jI > 0.0 && Bnu > 0.0) {
        const double iB = em1 * (1.0 / kSrcFac) * inu2 * inu;   // 1 / B_nu
        out[3] = jI * iB;
        out[4] = jQ * iB;
        out[5] = jV * iB;
        return out[3] > 0.0 ? seq : 0.0;
    }
    return 0.0;
}

// ---------------------------------------------------------------------------
// Exact constant-coefficient update of dS/dl = J - K S over w for thermal
// coefficients (J = S_eq (A_I, A_Q, 0, A_V), Kirchhoff).  K = A_I 1 + K' with
// K' a Lorentz-algebra generator (boost part (A_Q, 0, A_V), rotation part
// (R_Q, 0, R_V)).  With G = -K' w, whose eigenvalues are +-x and +-i y,
//   x^2 - y^2 = w^2 (|a|^2 - |r|^2),  x y = w^2 |a.r|,
// exp(-K w) = e^-tau (c0 + c1 G + c2 G^2 + c3 G^3), tau = A_I w,
//   c0 = (y^2 cosh x + x^2 cos y)/(x^2+y^2), c1 = (y^2 sinh x/x + x^2 sin y/y)/(x^2+y^2),
//   c2 = (cosh x - cos y)/(x^2+y^2),           c3 = (sinh x/x - sin y/y)/(x^2+y^2)
// (series forms for small x^2 + y^2).  The update is written as
//   S' = d0 S + (1 - d0) S_eq e0 + G (d1 D + G (d2 D + G d3 D)), D = S - S_eq e0,
// d_k = e^-tau c_k, with 1 - d0 = -expm1(-tau) + e^-tau (1 - c0) free of
// cancellation.
// ---------------------------------------------------------------------------
// G v with G = -w K'; K' rows (0, AQ, 0, AV), (AQ, 0, RV, 0), (0, -RV, 0, RQ), (AV, 0, -RQ, 0);
// called with the w-scaled entries gQ = -w AQ, gV = -w AV, hQ = -w RQ, hV = -w RV.
KRT_HD void gen_apply(double gQ, double gV, double hQ, double hV, const double v[4], double o[4]) {
    o[0] = gQ * v[1] + gV * v[3];
    o[1] = gQ * v[0] + hV * v[2];
    o[2] = hQ * v[3] - hV * v[1];
    o[3] = gV * v[0] - hQ * v[2];
}

// 1/n! for n = 0..21 (correctly rounded).
constexpr double kInvFact[22] = {
    1.0, 1.0, 0.5, 0.16666666666666666, 0.041666666666666664, 0.008333333333333333,
    0.001388888888888889, 0.0001984126984126984, 2.48015873015873e-05, 2.7557319223985893e-06,
    2.755731922398589e-07, 2.505210838544172e-08, 2.08767569878681e-09, 1.6059043836821613e-10,
    1.1470745597729725e-11, 7.647163731819816e-13, 4.779477332387385e-14, 2.8114572543455206e-15,
    1.5619206968586225e-16, 8.22063524662433e-18, 4.110317623312165e-19, 1.9572941063391263e-20};

KRT_HD void mueller_thermal(double Seq, double AI, double AQ, double AV, double RQ, double RV,
                            double w, double S[4]) {
    const double tau = AI * w;
    // invariants of K' (w-scaled)
    const double a2 = (AQ * AQ + AV * AV) * w * w;
    const double r2 = (RQ * RQ + RV * RV) * w * w;
    const double ar = (AQ * RQ + AV * RV) * w * w;
    const double q = 0.5 * (a2 - r2);
    const double rad = sqrt_fast(q * q + ar * ar);
    double X, Y;  // x^2 and y^2
    // (the smaller invariant is at most the larger one: below 1e-290 it is
    // taken as 0, which keeps the hardware reciprocal off subnormal inputs)
    if (q >= 0.0) {
        X = rad + q;
        Y = (X > 1e-290) ? ar * ar * rcp_fast(X) : 0.0;
    } else {
        Y = rad - q;
        X = (Y > 1e-290) ? ar * ar * rcp_fast(Y) : 0.0;
    }
    double d0, omd0, d1, d2, d3;
    const double XY = X + Y;
    if (XY < 0.1) {
        // series in X and Z = -Y: c2 = sum_k h_k/(2k)!, c3 = sum_k h_k/(2k+1)!,
        // c0 = 1 - X Z sum_{k>=1} h_k/(2k+2)!, c1 = 1 - X Z sum_{k>=1} h_k/(2k+3)!,
        // h_k = sum_{j<k} X^j Z^(k-1-j) (h_1 = 1, h_{k+1} = X h_k + Z^k).
        const double em1 = expm1_small(-tau);
        const double et = 1.0 + em1;
        const double Z = -Y;
        double h = 1.0, zk = 1.0;
        double c2 = 0.0, c3 = 0.0, s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int k = 1; k <= 9; ++k) {
            c2 += h * kInvFact[2 * k];
            c3 += h * kInvFact[2 * k + 1];
            s0 += h * kInvFact[2 * k + 2];
            s1 += h * kInvFact[2 * k + 3];
            zk *= Z;
            h = X * h + zk;
        }
        const double XZ = X * Z;
        d0 = et * (1.0 - XZ * s0);
        omd0 = -em1 + et * XZ * s0;
        d1 = et * (1.0 - XZ * s1);
        d2 = et * c2;
        d3 = et * c3;
    } else {
        // x = sqrt X and 1/x from one reciprocal square root (same for y);
        // below 1e-200 the invariant is taken as 0 (x < 1e-100 changes no term)
        const double rX = X > 1e-200 ? rsqrt_fast(X) : 0.0, rY = Y > 1e-200 ? rsqrt_fast(Y) : 0.0;
        const double x = X * rX, y = Y * rY;
        // u = e^((x - tau)/2), v = e^(-(x + tau)/2): e^(x-tau) = u^2,
        // e^(-x-tau) = v^2, e^-tau = u v
        const double u = exp(0.5 * (x - tau)), v = exp(-0.5 * (x + tau));
        const double ep = u * u, em = v * v, et = u * v;
        const double ch = 0.5 * (ep + em);                              // e^-tau cosh x
        const double shx = (x > 1e-8) ? 0.5 * (ep - em) * rX : et;  // e^-tau sinh x / x
        double sy, cy;
        sincos(y, &sy, &cy);
        const double syy = (y > 1e-8) ? sy * rY : 1.0;
        const double iXY = rcp_fast(XY);
        d0 = (Y * ch + X * et * cy) * iXY;
        d1 = (Y * shx + X * et * syy) * iXY;
        d2 = (ch - et * cy) * iXY;
        d3 = (shx - et * syy) * iXY;
        // e^-tau (1 - c0) = (2 X e^-tau sin^2(y/2) - 2 Y (e^-tau/2 sinh(x/2))^2) / (X + Y),
        // sin^2(y/2) = sin^2 y / (2 (1 + cos y)) (cos y > 0) or (1 - cos y) / 2
        const double qh = 0.5 * (u - v);
        const double s2h = (cy > 0.0) ? 0.5 * sy * sy * rcp_fast(1.0 + cy) : 0.5 * (1.0 - cy);
        omd0 = -expm1_small(-tau) + 2.0 * (X * et * s2h - Y * qh * qh) * iXY;
    }
    double D[4] = {S[0] - Seq, S[1], S[2], S[3]};
    double T[4], U[4];
    const double gQ = -w * AQ, gV = -w * AV, hQ = -w * RQ, hV = -w * RV;
    for (int k = 0; k < 4; ++k) T[k] = d3 * D[k];
    gen_apply(gQ, gV, hQ, hV, T, U);
    for (int k = 0; k < 4; ++k) T[k] = d2 * D[k] + U[k];
    gen_apply(gQ, gV, hQ, hV, T, U);
    for (int k = 0; k < 4; ++k) T[k] = d1 * D[k] + U[k];
    gen_apply(gQ, gV, hQ, hV, T, U);
    S[0] = d0 * S[0] + omd0 * Seq + U[0];
    S[1] = d0 * S[1] + U[1];
    S[2] = d0 * S[2] + U[2];
    S[3] = d0 * S[3] + U[3];
}

// ---------------------------------------------------------------------------
// Coherency matrix N = NR + i NI (NR symmetric: 10 entries, NI antisymmetric:
// 6 entries), packed upper triangles.
// ---------------------------------------------------------------------------
struct Coh {
    double R[10];  // (00,01,02,03,11,12,13,22,23,33)
    double I[6];   // (01,02,03,12,13,23)
};

KRT_HD constexpr int sym_idx(int i, int j) {
    return (i <= j) ? (i * 4 - (i * (i - 1)) / 2 + (j - i)) : (j * 4 - (j * (j - 1)) / 2 + (i - j));
}
KRT_HD constexpr int asym_idx(int i, int j) {  // i < j
    return (i == 0) ? (j - 1) : ((i == 1) ? (j + 1) : 5);
}
KRT_HD double nr(const Coh& N, int i, int j) { return N.R[sym_idx(i, j)]; }
KRT_HD double ni(const Coh& N, int i, int j) {
    return (i == j) ? 0.0 : ((i < j) ? N.I[asym_idx(i, j)] : -N.I[asym_idx(j, i)]);
}

// F(A, N) = -(A N + N A^T), entry by entry as one chain of fused
// multiply-adds over the non-zero terms (the imaginary part has a zero
// diagonal); the chain starts from its first product, not from 0.
KRT_HD void transport_rhs(const double A[16], const Coh& N, Coh& F) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = i; j < 4; ++j) {
            double s = A[i * 4] * nr(N, 0, j);
            s = fma(nr(N, i, 0), A[j * 4], s);
#pragma unroll
            for (int b = 1; b < 4; ++b) {
                s = fma(A[i * 4 + b], nr(N, b, j), s);
                s = fma(nr(N, i, b), A[j * 4 + b], s);
            }
            F.R[sym_idx(i, j)] = -s;
        }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = i + 1; j < 4; ++j) {
            // A_ib N_bj (b != j) + N_ib A_jb (b != i); the first term is b = 0
            // or, for i = 0, b = 1 (j >= 1, so b = 0 != j)
            double s = A[i * 4] * ni(N, 0, j);
#pragma unroll
            for (int b = 1; b < 4; ++b)
                if (b != j) s = fma(A[i * 4 + b], ni(N, b, j), s);
#pragma unroll
            for (int b = 0; b < 4; ++b)
                if (b != i) s = fma(ni(N, i, b), A[j * 4 + b], s);
            F.I[asym_idx(i, j)] = -s;
        }
}

// Stokes of N on two legs given as covectors l1, l2:
// I = N11 + N22, Q = N11 - N22, U = 2 Re N12, V = -2 Im N12.
KRT_HD void coh_project(const Coh& N, const double l1[4], const double l2[4], double S[4]) {
    double n11 = 0.0, n22 = 0.0, n12 = 0.0, m12 = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        double y1 = 0.0, y2 = 0.0, z2 = 0.0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            y1 += nr(N, i, j) * l1[j];
            y2 += nr(N, i, j) * l2[j];
            if (j != i) z2 += ni(N, i, j) * l2[j];
        }
        n11 += l1[i] * y1;
        n12 += l1[i] * y2;
        n22 += l2[i] * y2;
        m12 += l1[i] * z2;
    }
    S[0] = n11 + n22;
    S[1] = n11 - n22;
    S[2] = 2.0 * n12;
    S[3] = -2.0 * m12;
}

// N from Stokes on two legs given as vectors e1, e2.
// N = n11 e1 e1 + n22 e2 e2 + nre (e1 e2 + e2 e1) + i nim (e1 e2 - e2 e1),
// as N^ij = e1^i p^j + e2^i q^j with p = n11 e1 + nre e2, q = n22 e2 + nre e1.
KRT_HD void coh_rebuild(Coh& N, const double S[4], const double e1[4], const double e2[4]) {
    const double n11 = 0.5 * (S[0] + S[1]), n22 = 0.5 * (S[0] - S[1]);
    const double nre = 0.5 * S[2], nim = -0.5 * S[3];
    double p[4], q[4], r1[4], r2[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        p[j] = n11 * e1[j] + nre * e2[j];
        q[j] = n22 * e2[j] + nre * e1[j];
        r1[j] = nim * e1[j];
        r2[j] = nim * e2[j];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = i; j < 4; ++j) N.R[sym_idx(i, j)] = e1[i] * p[j] + e2[i] * q[j];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = i + 1; j < 4; ++j) N.I[asym_idx(i, j)] = e1[i] * r2[j] - e2[i] * r1[j];
}

// ---------------------------------------------------------------------------
// Fluid tetrad legs e1, e2 (contravariant and covariant): e0 = u,
// e3 = unit vector along K + (K.u) u (the photon direction in the fluid
// frame; (K + (K.u) u)/(-K.u) for exactly null K), e2 along the part of b
// orthogonal to u and e3
// (fallback d_theta, then d_r), e1 from the Levi-Civita tensor so that
// (e0, e1, e2, e3) is right-handed: e1_nu = eps_{mu nu rho sigma} e0^mu e2^rho e3^sigma.
// ---------------------------------------------------------------------------
KRT_HD double det3(double a0, double a1, double a2, double b0, double b1, double b2, double c0,
                   double c1, double c2) {
    return a0 * (b1 * c2 - b2 * c1) - a1 * (b0 * c2 - b2 * c0) + a2 * (b0 * c1 - b1 * c0);
}

KRT_HD void fluid_legs(const Metric& g, const double u[4], const double K[4], const double b[4],
                       double bb, double Ku, double e1[4], double l1[4], double e2[4], double l2[4]) {
    double e3[4], l3[4], ul[4];
    for (int k = 0; k < 4; ++k) e3[k] = K[k] + Ku * u[k];
    lower(g, e3, l3);
    const double i3 = rsqrt_fast(e3[0] * l3[0] + e3[1] * l3[1] + e3[2] * l3[2] + e3[3] * l3[3]);
    for (int k = 0; k < 4; ++k) {
        e3[k] *= i3;
        l3[k] *= i3;
    }
    lower(g, u, ul);
    // candidate along b
    double v[4];
    {
        const double bu = b[0] * ul[0] + b[1] * ul[1] + b[2] * ul[2] + b[3] * ul[3];
        const double b3 = b[0] * l3[0] + b[1] * l3[1] + b[2] * l3[2] + b[3] * l3[3];
        for (int k = 0; k < 4; ++k) v[k] = b[k] + bu * u[k] - b3 * e3[k];
    }
    double vv = dot(g, v, v);
    // |v| >= 1e-10 |b| tested in squares (no square roots on the common path)
    if (!(bb > 0.0) || !(vv >= 1e-20 * bb)) {
        double vn;
        for (int c = 0; c < 2; ++c) {
            const int dir = (c == 0) ? 2 : 1;
            const double cn = sqrt_fast(dir == 2 ? g.hh : g.rr);
            const double pu = ul[dir], p3 = l3[dir];
            for (int k = 0; k < 4; ++k) v[k] = ((k == dir) ? 1.0 : 0.0) + pu * u[k] - p3 * e3[k];
            vv = dot(g, v, v);
            vn = vv > 0.0 ? sqrt_fast(vv) : 0.0;
            if (vn >= 1e-10 * cn) break;
        }
    }
    const double iv = vv > 0.0 ? rsqrt_fast(vv) : __builtin_inf();
    for (int k = 0; k < 4; ++k) e2[k] = v[k] * iv;
    lower(g, e2, l2);
    // e1_nu from the Levi-Civita tensor, sqrt(-g) = Sigma sin(theta)
    const double sg = g.Sig * g.s;
    const double* P = u;
    const double* Q = e2;
    const double* R = e3;
    l1[0] = -sg * det3(P[1], P[2], P[3], Q[1], Q[2], Q[3], R[1], R[2], R[3]);
    l1[1] = sg * det3(P[0], P[2], P[3], Q[0], Q[2], Q[3], R[0], R[2], R[3]);
    l1[2] = -sg * det3(P[0], P[1], P[3], Q[0], Q[1], Q[3], R[0], R[1], R[3]);
    l1[3] = sg * det3(P[0], P[1], P[2], Q[0], Q[1], Q[2], R[0], R[1], R[2]);
    raise(g, l1, e1);
}

}  // namespace krt
