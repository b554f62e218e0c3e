// Nonthermal (kappa) electrons: synchrotron coefficients by integration over
// the Lorentz factor, and the constant-coefficient Stokes update for a
// general (non-Kirchhoff) emissivity.
//
// The paper (Sec. 2.1, Sec. 4) names the electron distribution among the
// model inputs and nonthermal electrons as the extension; the formulae are
// those of standard synchrotron theory, read as follows (the same readings
// as the CPU oracle, written independently):
//  - distribution, normalised to one electron, isotropic in pitch angle:
//      N(g) = A g sqrt(g^2-1) (1 + (g-1)/(kappa w))^-(kappa+1);
//  - per-electron emission at angle theta to the field: c0 F(Xg) (I),
//    c0 G(Xg) (Q), c0 (4/3) cot(theta) H(Xg) / g (V), with
//    c0 = sqrt3 e^3 B sin(theta) / (4 pi m c^2), Xg = X w^2 / g^2,
//    X = nu / nu_c, nu_c = 1.5 nu_B sin(theta) w^2,
//    F = X int_X K_5/3, G = X K_2/3, H = X K_1/3 + int_X K_1/3;
//  - absorption from the Einstein relation of an isotropic distribution,
//    alpha_S = (1 / (2 nu^2 m_e)) int P_S D dg, D = -g sqrt(g^2-1)
//    d/dg [N / (g sqrt(g^2-1))] = N (kappa+1) / (kappa w q), q = 1 + (g-1)/(kappa w);
//  - rotativities: weights acosh(g) / (g sqrt(g^2-1)) (rho_V) and
//    (2g - 1/g) Xg / (1 + Xg) (rho_Q), with the thermal prefactors.
// The eight dimensionless integrals (I_F, I_G, I_H, A_F, A_G, A_H, R_Q, R_V)
// depend on (kappa, w, X) only.
#pragma once

#include <type_traits>
#include "krt_device.hpp"

namespace krt {

// ---------------------------------------------------------------------------
// Synchrotron functions F, G, H: table of ln(F e^X), ln(G e^X), ln(H e^X) in
// s = ln X over [ln 1e-16, ln 700], kSynPanels Chebyshev panels of degree
// kSynDeg, built once per context from the integral representations
// K_nu(x) = int_0^inf exp(-x cosh t) cosh(nu t) dt and
// int_x^inf K_nu = int_0^inf exp(-x cosh t) cosh(nu t) / cosh t dt.
// ---------------------------------------------------------------------------
constexpr int kSynPanels = 96;
constexpr int kSynDeg = 15;
constexpr int kSynCoef = kSynDeg + 1;
constexpr double kSynS0 = -36.841361487904734;  // ln 1e-16
constexpr double kSynS1 = 6.551080335043404;    // ln 700
constexpr int kSynTab = kSynPanels * 3 * kSynCoef;

// e^x K_nu(x) and e^x int_x^inf K_nu by the trapezoid rule (the integrands
// are even and entire in t, so the rule converges geometrically); the range
// ends where x (cosh T - 1) - nu T >= 45.
KRT_HD void syn_reps(double nu, double x, double& k, double& ki) {
    double T = 1.0;
    for (int it = 0; it < 8; ++it) T = acosh(1.0 + (45.0 + nu * T) / x);
    const double h = fmin(0.1, 0.5 / sqrt(x));
    const int ns = (int)ceil(T / h);
    double sk = 0.5, ski = 0.5;
    for (int q = 1; q <= ns; ++q) {
        const double t = q * h;
        const double ch = cosh(t);
        const double e = exp(-x * (ch - 1.0)) * cosh(nu * t);
        sk += e;
        ski += e / ch;
    }
    k = sk * h;
    ki = ski * h;
}

__global__ void syn_table_nodes(double* vals) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= kSynPanels * kSynCoef) return;
    const int p = idx / kSynCoef, k = idx % kSynCoef;
    const double width = (kSynS1 - kSynS0) / kSynPanels;
    const double z = cos(kPi * (k + 0.5) / kSynCoef);
    const double x = exp(kSynS0 + (p + 0.5) * width + 0.5 * width * z);
    double k13, ki13, k23, ki23, k53, ki53;
    syn_reps(1.0 / 3.0, x, k13, ki13);
    syn_reps(2.0 / 3.0, x, k23, ki23);
    syn_reps(5.0 / 3.0, x, k53, ki53);
    vals[idx * 3 + 0] = log(x * ki53);
    vals[idx * 3 + 1] = log(x * k23);
    vals[idx * 3 + 2] = log(x * k13 + ki13);
}

__global__ void syn_table_coefs(const double* vals, double* table) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= kSynTab) return;
    const int p = idx / (3 * kSynCoef), f = (idx / kSynCoef) % 3, j = idx % kSynCoef;
    double s = 0.0;
    for (int k = 0; k < kSynCoef; ++k) s += vals[(p * kSynCoef + k) * 3 + f] * cos(kPi * j * (k + 0.5) / kSynCoef);
    s *= 2.0 / kSynCoef;
    if (j == 0) s *= 0.5;
    table[idx] = s;
}

// Small-argument forms: F -> (4 pi / (sqrt3 Gamma(1/3))) (X/2)^(1/3), G -> F/2,
// H -> pi / sqrt3 (relative error ~ X^(2/3), below 3e-11 for X < 1e-16).
constexpr double kSynF0 = 2.1495282415344787;   // 4 pi / (sqrt3 Gamma(1/3)) 2^(-1/3)
constexpr double kSynH0 = 1.8137993642342178;   // pi / sqrt3

KRT_HD void syn_functions(const double* __restrict__ tab, double X, double& F, double& G, double& H) {
    if (!(X <= 700.0)) {
        F = G = H = 0.0;
        return;
    }
    if (X < 1e-16) {
        F = kSynF0 * cbrt(X);
        G = 0.5 * F;
        H = kSynH0;
        return;
    }
    const double width = (kSynS1 - kSynS0) / kSynPanels;
    const double s = log(X);
    int p = (int)((s - kSynS0) * (1.0 / width));
    p = p < 0 ? 0 : (p >= kSynPanels ? kSynPanels - 1 : p);
    const double z = (2.0 * (s - kSynS0) - (2 * p + 1) * width) * (1.0 / width);
    const double* c = tab + (size_t)p * 3 * kSynCoef;
    double v[3];
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        // Clenshaw
        double b1 = 0.0, b2 = 0.0;
        for (int j = kSynDeg; j >= 1; --j) {
            const double b0 = 2.0 * z * b1 - b2 + c[f * kSynCoef + j];
            b2 = b1;
            b1 = b0;
        }
        v[f] = z * b1 - b2 + c[f * kSynCoef];
    }
    F = exp(v[0] - X);
    G = exp(v[1] - X);
    H = exp(v[2] - X);
}

// ---------------------------------------------------------------------------
// The eight dimensionless integrals by the trapezoid rule in u = ln(g - 1)
// over [-20, 25] with step 1/8 (analytic integrands, negligible at both ends:
// the rule converges geometrically; 1e-10 of the step-0.05 result).
// ---------------------------------------------------------------------------
constexpr int kKapNodes = 361;
constexpr double kKapU0 = -20.0;
constexpr double kKapDu = 0.125;

// Contribution of quadrature node i to the normalisation and the eight sums.
KRT_HD void kappa_node(const double* __restrict__ syntab, double kap, double w, double X, int i, double& norm,
                       double acc[8]) {
    const double ikw = 1.0 / (kap * w);
    const double kp1 = kap + 1.0;
    const double Xw2 = X * w * w;
    {
        const double gm1 = exp(kKapU0 + kKapDu * i);
        const double g = 1.0 + gm1;
        const double p = sqrt(gm1 * (g + 1.0));
        const double lq = log1p(gm1 * ikw);
        const double f = g * p * gm1 * exp(-kp1 * lq);   // N(g) dg/du, up to A
        const double d = f * kp1 * ikw * exp(-lq);
        norm += f;
        const double ig = 1.0 / g;
        const double Xg = Xw2 * ig * ig;
        double Fv, Gv, Hv;
        syn_functions(syntab, Xg, Fv, Gv, Hv);
        acc[0] += f * Fv;
        acc[1] += f * Gv;
        acc[2] += f * Hv * ig;
        acc[3] += d * Fv;
        acc[4] += d * Gv;
        acc[5] += d * Hv * ig;
        acc[6] += f * (2.0 * g - ig) * (Xg / (1.0 + Xg));
        acc[7] += f * log1p(gm1 + p) * ig / p;
    }
}

KRT_HD void kappa_integrals(const double* __restrict__ syntab, double kap, double w, double X, double o[8]) {
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    double norm = 0.0;
    for (int i = 0; i < kKapNodes; ++i) kappa_node(syntab, kap, w, X, i, norm, acc);
    const double in = 1.0 / norm;
#pragma unroll
    for (int k = 0; k < 8; ++k) o[k] = acc[k] * in;
}

// The same integrals for one point, computed by a whole wave: lane l takes
// the nodes l, l + 64, ..., and the nine sums are reduced across the wave.
// Every lane passes the same (kap, w, X) and gets the result.  Must be called
// by all 64 lanes together.
__device__ __forceinline__ void kappa_integrals_wave(const double* __restrict__ syntab, double kap, double w,
                                                     double X, double o[8]) {
    const int lane = threadIdx.x & 63;
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    double norm = 0.0;
    for (int i = lane; i < kKapNodes; i += 64) kappa_node(syntab, kap, w, X, i, norm, acc);
    for (int off = 32; off >= 1; off >>= 1) {
        norm += __shfl_xor(norm, off);
        for (int k = 0; k < 8; ++k) acc[k] += __shfl_xor(acc[k], off);
    }
    const double in = 1.0 / norm;
    for (int k = 0; k < 8; ++k) o[k] = acc[k] * in;
}

// Fluid-frame coefficients (cgs, layout of thermal_coefficients) from the
// dimensionless integrals I at (kappa, w, X(nu, B, theta)); guards as in the
// thermal module: no plasma gives zeros, sin(theta) < 1e-10 keeps rho_V only,
// polarized emissivity and absorptivity clamped to the total ones.
constexpr double kKapC0 = 1.7320508075688772 * kE * kE * kE / (4.0 * kPi * kME * kC * kC);

KRT_HD bool kappa_frame(double ne, double w, double B, double nu, double cth, double& X, double& sth) {
    if (!(ne > 0.0) || !(w > 0.0) || !(B > 0.0) || !(nu > 0.0)) return false;
    cth = cth > 1.0 ? 1.0 : (cth < -1.0 ? -1.0 : cth);
    sth = sqrt_fast(1.0 - cth * cth);
    const double nuc = 1.5 * kNuBPerB * B * sth * w * w;
    X = (nuc > 1e-290) ? nu * rcp_fast(nuc) : 1e300;
    if (!(X < 1e300)) X = 1e300;
    return true;
}

KRT_HD void kappa_physical(const double I[8], double ne, double B, double nu, double cth, double sth,
                           double out[8]) {
    cth = cth > 1.0 ? 1.0 : (cth < -1.0 ? -1.0 : cth);
    const double nuB = kNuBPerB * B;
    const double inu = rcp_fast(nu);
    out[7] = kRhoVFac * ne * nuB * cth * inu * inu * I[7];
    if (sth < 1e-10) {
        for (int k = 0; k < 7; ++k) out[k] = 0.0;
        return;
    }
    out[6] = 0.5 * kRhoVFac * ne * nuB * nuB * sth * sth * inu * inu * inu * I[6];
    const double pre = ne * kKapC0 * B * sth;
    const double cv = (4.0 / 3.0) * cth * rcp_fast(sth);
    double jI = pre * I[0], jQ = pre * I[1], jV = pre * cv * I[2];
    const double ab = 0.5 * inu * inu / kME;
    double aI = pre * ab * I[3], aQ = pre * ab * I[4], aV = pre * ab * cv * I[5];
    // clamp |j_P| <= j_I and |a_P| <= a_I, compared in squares where they
    // stay normal numbers (hypot elsewhere)
    const bool sqj = jI > 1e-140 && jI < 1e140, sqa = aI > 1e-140 && aI < 1e140;
    if (sqj ? (jQ * jQ + jV * jV > jI * jI) : (hypot(jQ, jV) > jI)) {
        const double sc = jI / hypot(jQ, jV);
        jQ *= sc;
        jV *= sc;
    }
    if (sqa ? (aQ * aQ + aV * aV > aI * aI) : (hypot(aQ, aV) > aI)) {
        const double sc = aI / hypot(aQ, aV);
        aQ *= sc;
        aV *= sc;
    }
    out[0] = jI;
    out[1] = jQ;
    out[2] = jV;
    out[3] = aI;
    out[4] = aQ;
    out[5] = aV;
}

// ---------------------------------------------------------------------------
// Exact constant-coefficient update of dS/dl = J - K S over w for a general
// emissivity J = (J_I, J_Q, 0, J_V):
//   S' = exp(-K w) S + w phi1(-K w) J,   phi1(z) = (e^z - 1) / z.
// With K = A_I + K' and G = -w K' (eigenvalues +-x, +-i y), any f(-tau + G)
// is the cubic a0 + a1 G + a2 G^2 + a3 G^3 interpolating f(-tau + lambda) at
// the four eigenvalues:  with f_e, f_o the even part and odd part / lambda,
//   a2 = (f_e(x) - f_e(iy)) / (x^2+y^2), a0 = (y^2 f_e(x) + x^2 f_e(iy)) / (x^2+y^2),
//   a3 = (f_o(x) - f_o(iy)) / (x^2+y^2), a1 = (y^2 f_o(x) + x^2 f_o(iy)) / (x^2+y^2);
// for small x^2+y^2 (or small x^2, y^2) the same from the Taylor coefficients
// t_n = f^(n)(-tau) / n!.  exp(-K w) uses the thermal module's coefficients.
// ---------------------------------------------------------------------------
// Taylor coefficients of phi1 at z = -tau <= 0: t_n = int_0^1 e^(z s) s^n / n! ds
// = e^z sum_k tau^k / (n+k+1)!, linked by t_(n-1) = e^z / n! + tau t_n.  The
// recurrence is used where it is stable: upward, t_n = (t_(n-1) - e^z/n!) / tau,
// for n <= tau; downward for n > tau, from a start n0 far enough above 21
// where t_n0 is taken as e^z / ((n0+1)! (1 - tau/(n0+2))) (the error this
// start leaves is damped by tau/n per step).  Relative error a few ulp for
// every tau >= 0.
constexpr double kInvFact81 = 1.724992688482352e-121;   // 1/81!

// e^-z t_21 by the downward recurrence in scaled form, s_(n-1) = 1/n! + tau s_n,
// from s_n0 = 1 / ((n0+1)! (1 - tau/(n0+2))).  The start's relative error,
// about (tau/n0)^2, is damped by tau/n per step: n0 = 32 for tau < 1 leaves
// below 1e-19 at n = 21, n0 = 80 covers tau < 21 (where the downward values
// are used).
constexpr double kInvFact33 = 1.151633562077195e-37;   // 1/33!
KRT_HD double phi1_tail_scaled(double tau) {
    const bool low = tau < 1.0;
    const int n0 = low ? 32 : 80;
    const double inv = low ? kInvFact33 : kInvFact81;   // 1/(n0+1)!
    double f = inv * (double)(n0 + 1);                  // 1/n0!
    double s = inv / (1.0 - tau / (double)(n0 + 2));
    for (int n = n0; n >= 22; --n) {
        s = f + tau * s;                                 // s_(n-1)
        f *= (double)n;
    }
    return s;
}

// Storage of a lane's 22 coefficients in LDS (entry n at p[64 n]: the
// lanes of a wave side by side), for kernels without registers to hold them.
struct LdsLaneTab {
    volatile __attribute__((address_space(3))) double* p;
    __device__ __forceinline__ volatile __attribute__((address_space(3))) double& operator[](int n) const {
        return p[n << 6];
    }
};

// t: double[22] or LdsLaneTab.
template <class Tab>
KRT_HD void phi1_taylor(double z, double em1, Tab& t) {
    // em1 = e^z - 1 from the caller
    const double tau = -z;
    const double ez = 1.0 + em1;
    t[0] = (tau > 1e-200) ? em1 * rcp_fast(z) : 1.0;
    if constexpr (std::is_array<Tab>::value) {
        // a register table: fixed indices only.  Downward for every tau, the
        // values at n <= tau replaced by the upward ones
        t[21] = ez * phi1_tail_scaled(tau);
#pragma unroll
        for (int n = 21; n >= 2; --n) t[n - 1] = ez * kInvFact[n] + tau * t[n];
        if (tau >= 1.0) {
            const int m = tau >= 21.0 ? 21 : (int)tau;
            const double it = 1.0 / tau;
            double u = t[0];
#pragma unroll
            for (int n = 1; n <= 21; ++n) {
                u = (u - ez * kInvFact[n]) * it;
                if (n <= m) t[n] = u;
            }
        }
    } else {
        // a table in memory: each entry computed once
        int m = 0;
        if (tau >= 1.0) {
            m = tau >= 21.0 ? 21 : (int)tau;
            const double it = 1.0 / tau;
            for (int n = 1; n <= m; ++n) t[n] = (t[n - 1] - ez * kInvFact[n]) * it;
        }
        if (m < 21) {
            double tn = ez * phi1_tail_scaled(tau);            // t_21
            t[21] = tn;
            for (int n = 21; n >= m + 2; --n) {
                tn = ez * kInvFact[n] + tau * tn;
                t[n - 1] = tn;
            }
        }
    }
}

// phi1 at a real z <= 0.
KRT_HD double phi1_real(double z) { return (z == 0.0) ? 1.0 : expm1(z) / z; }

template <class Tab>
KRT_HD void mueller_general(double JI, double JQ, double JV, double AI, double AQ, double AV, double RQ,
                            double RV, double w, double S[4], Tab& t) {
    const double tau = AI * w;
    const double a2 = (AQ * AQ + AV * AV) * w * w;
    const double r2 = (RQ * RQ + RV * RV) * w * w;
    const double ar = (AQ * RQ + AV * RV) * w * w;
    const double q = 0.5 * (a2 - r2);
    const double rad = sqrt(q * q + ar * ar);
    double X, Y;
    if (q >= 0.0) {
        X = rad + q;
        Y = (X > 0.0) ? ar * ar / X : 0.0;
    } else {
        Y = rad - q;
        X = (Y > 0.0) ? ar * ar / Y : 0.0;
    }
    const double XY = X + Y;
    const double Z = -Y;
    const double em1 = expm1_small(-tau);
    const double et = 1.0 + em1;
    phi1_taylor(-tau, em1, t);
    // exp(-K w) = d0 + d1 G + d2 G^2 + d3 G^3 and phi1(-K w) = b0 + b1 G + b2 G^2 + b3 G^3
    double d0, d1, d2, d3, b0, b1, b2, b3;
    if (XY < 0.1) {
        double h = 1.0, hprev = 0.0, zk = 1.0;
        double c2 = 0.0, c3 = 0.0, s0 = 0.0, s1 = 0.0;
        double u0 = 0.0, u1 = 0.0, u2 = 0.0, u3 = 0.0;
        for (int k = 1; k <= 10; ++k) {
            if (k <= 9) {
                c2 += h * kInvFact[2 * k];
                c3 += h * kInvFact[2 * k + 1];
                s0 += h * kInvFact[2 * k + 2];
                s1 += h * kInvFact[2 * k + 3];
            }
            // phi1: G^(2k) = -X Z h_(k-1) + h_k G^2
            u0 += t[2 * k] * hprev;
            u2 += t[2 * k] * h;
            if (2 * k + 1 < 22) {
                u1 += t[2 * k + 1] * hprev;
                u3 += t[2 * k + 1] * h;
            }
            hprev = h;
            zk *= Z;
            h = X * h + zk;
        }
        const double XZ = X * Z;
        d0 = et * (1.0 - XZ * s0);
        d1 = et * (1.0 - XZ * s1);
        d2 = et * c2;
        d3 = et * c3;
        b0 = t[0] - XZ * u0;
        b1 = t[1] - XZ * u1;
        b2 = u2;
        b3 = u3;
    } else {
        const double x = sqrt_fast(X), y = sqrt_fast(Y);
        const double u = exp(0.5 * (x - tau)), v = exp(-0.5 * (x + tau));
        const double ep = u * u, emx = v * v;
        const double ch = 0.5 * (ep + emx);
        const double shx = (x > 1e-8) ? 0.5 * (ep - emx) / x : et;
        double sy, cy;
        sincos(y, &sy, &cy);
        const double syy = (y > 1e-8) ? sy / y : 1.0;
        const double iXY = 1.0 / XY;
        d0 = (Y * ch + X * et * cy) * iXY;
        d1 = (Y * shx + X * et * syy) * iXY;
        d2 = (ch - et * cy) * iXY;
        d3 = (shx - et * syy) * iXY;
        // even and odd parts of phi1(-tau + lambda) at lambda = x and i y
        double fex, fox, fey, foy;
        if (X < 0.01) {
            fex = fox = 0.0;
            double xp = 1.0;
            for (int k = 0; k <= 9; ++k) {
                fex += t[2 * k] * xp;
                fox += t[2 * k + 1] * xp;
                xp *= X;
            }
        } else {
            const double pp = phi1_real(-tau + x), pm = phi1_real(-tau - x);
            fex = 0.5 * (pp + pm);
            fox = 0.5 * (pp - pm) / x;
        }
        if (Y < 0.01) {
            fey = foy = 0.0;
            double yp = 1.0;
            for (int k = 0; k <= 9; ++k) {
                fey += t[2 * k] * yp;
                foy += t[2 * k + 1] * yp;
                yp *= Z;
            }
        } else {
            // phi1(-tau + i y) = (e^-tau e^(iy) - 1) / (-tau + i y)
            const double sh = sin(0.5 * y);
            const double nr = em1 * cy - 2.0 * sh * sh;   // e^-tau cos y - 1
            const double ni = et * sy;
            const double den = 1.0 / (tau * tau + Y);
            fey = (-tau * nr + y * ni) * den;
            foy = (-tau * ni - y * nr) * den / y;
        }
        b2 = (fex - fey) * iXY;
        b0 = (Y * fex + X * fey) * iXY;
        b3 = (fox - foy) * iXY;
        b1 = (Y * fox + X * foy) * iXY;
    }
    // S' = (d0 + G(d1 + G(d2 + G d3))) S + w (b0 + G(b1 + G(b2 + G b3))) J
    const double J[4] = {JI * w, JQ * w, 0.0, JV * w};
    double T[4], U[4];
    const double gQ = -w * AQ, gV = -w * AV, hQ = -w * RQ, hV = -w * RV;
    for (int k = 0; k < 4; ++k) T[k] = d3 * S[k] + b3 * J[k];
    gen_apply(gQ, gV, hQ, hV, T, U);
    for (int k = 0; k < 4; ++k) T[k] = d2 * S[k] + b2 * J[k] + U[k];
    gen_apply(gQ, gV, hQ, hV, T, U);
    for (int k = 0; k < 4; ++k) T[k] = d1 * S[k] + b1 * J[k] + U[k];
    gen_apply(gQ, gV, hQ, hV, T, U);
    for (int k = 0; k < 4; ++k) S[k] = d0 * S[k] + b0 * J[k] + U[k];
}

KRT_HD void mueller_general(double JI, double JQ, double JV, double AI, double AQ, double AV, double RQ,
                            double RV, double w, double S[4]) {
    double t[22];
    mueller_general(JI, JQ, JV, AI, AQ, AV, RQ, RV, w, S, t);
}

}  // namespace krt
