// FP32 transfer operators with FP64 state (mixed-precision transfer).
//
// The geodesic and its stored path stay FP64.  At every stored point the
// operators of the transfer step -- metric and connection, plasma, thermal
// coefficients, fluid tetrad, propagator -- are formed in FP32; the
// coherency matrix N and the Heun transport state stay FP64, and every
// update (transport increment, radiative increment) is computed in FP32 and
// added to the FP64 state.  Invariant intensities are ~1e-48 in cgs, below
// the FP32 range, so they pass through the FP32 operators scaled by 2^160;
// frequency-dependent prefactors are folded with the camera frequency on the
// host in FP64 and the kernels work with the redshift factor g = nu / nu_cam.
#pragma once

#include "krt_device.hpp"

namespace krt {

constexpr double kIScale = 1.4615016373309029e48;     // 2^160
constexpr double kIScaleInv = 6.842277657836021e-49;  // 2^-160

// Per-launch constants, folded on the host in FP64 and rounded to FP32.
struct F32Consts {
    float a, m;      // spin, mass factor
    float cJ;        // e^2 nu_cam / (2 sqrt3 c): j_I = cJ n_e g I(x) / Theta^2
    float cRV;       // 2 e^2 / (m_e c nu_cam^2)
    float cRQ;       // e^2 / (m_e c nu_cam^3)
    float cHnu;      // h nu_cam / (m_e c^2): h nu / (k T_e) = cHnu g / Theta
    float cBnu;      // 2 h nu_cam^3 / c^2
    float cSeq;      // 2^160 * 2 h / c^2
    float nu_cam;
    float L;         // L_cm
    // analytic ADAF
    float n0, thr, cB2, ih2, risco;  // n_e scale, Theta_e r, B^2 = cB2 n_e / r, 1 / (2 h^2)
    // snapshot: grid origin and inverse spacing in x1, x2; hh = (1 - hslope)/2;
    // gamma_ad - 1; n_e per code density; B per code field; m_p / m_e
    float x1s, idx1, x2s, idx2, hh, gm1, ne_unit, B_unit, Rhigh, Rlow, sigma_cut, rmax, mpme;
};

// Reciprocal, square root and reciprocal square root on the FP32 units (about
// 1 ulp): the operators of this mode need no correctly rounded division or
// square root, whose expansions take 12 and 17 instructions.
KRT_HD float rcpf_fast(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.0f / x;
#endif
}
KRT_HD float sqrtf_fast(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_sqrtf(x);
#else
    return sqrtf(x);
#endif
}
KRT_HD float rsqrtf_fast(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rsqf(x);
#else
    return 1.0f / sqrtf(x);
#endif
}

// exp, log and expm1 from the hardware's base-2 exp and log (relative error
// about |x| 2^-24 plus an ulp, against the library's correctly reduced forms);
// x^(-1/3) from them with one Newton step.
KRT_HD float expf_fast(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_exp2f(x * 1.44269504f);
#else
    return expf(x);
#endif
}
KRT_HD float logf_fast(float x) {   // x > 0, normal
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_logf(x) * 0.693147181f;
#else
    return logf(x);
#endif
}
// Taylor series through x^6 for |x| < 1/8 (relative truncation below 1e-9).
KRT_HD float expm1f_fast(float x) {
    if (fabsf(x) < 0.125f)
        return x * (1.0f + x * (0.5f + x * (1.0f / 6.0f + x * (1.0f / 24.0f + x * (1.0f / 120.0f + x * (1.0f / 720.0f))))));
    return expf_fast(x) - 1.0f;
}
KRT_HD float rcbrtf_fast(float x) {   // x > 0, normal
#if defined(__HIP_DEVICE_COMPILE__)
    const float y = __builtin_amdgcn_exp2f(-0.333333343f * __builtin_amdgcn_logf(x));
    return y * (4.0f - x * y * y * y) * 0.333333343f;   // y (4 - x y^3) / 3
#else
    return 1.0f / cbrtf(x);
#endif
}
// sin and cos of 2 pi t for t in [-256, 256] (turns), on the hardware units.
KRT_HD void sincos_turns_f(float t, float& sn, float& cs) {
#if defined(__HIP_DEVICE_COMPILE__)
    sn = __builtin_amdgcn_sinf(t);
    cs = __builtin_amdgcn_cosf(t);
#else
    sincosf(6.28318531f * t, &sn, &cs);
#endif
}

struct MetricF {
    float s, c, Sig;
    float tt, tr, tp, rr, rp, hh, pp;
    float Itt, Itr, Irr, Irp, Ihh, Ipp;
};

struct MetricDF {
    float tt, tr, tp, rr, rp, hh, pp;
};

// Kerr-Schild metric, its r and theta derivatives and its inverse (same
// closed forms as the FP64 path).
KRT_HD void metric_d_f(float a, float m, float r, float s, float c, MetricF& g, MetricDF& dr,
                       MetricDF& dh) {
    const float s2 = s * s, sc = s * c, a2 = a * a;
    const float Sig = r * r + a2 * c * c;
    const float iS = rcpf_fast(Sig);
    const float f = 2.0f * m * r * iS;
    const float opf = 1.0f + f;
    g.s = s;
    g.c = c;
    g.Sig = Sig;
    g.tt = f - 1.0f;
    g.tr = f;
    g.tp = -a * f * s2;
    g.rr = opf;
    g.rp = -a * s2 * opf;
    g.hh = Sig;
    g.pp = s2 * (Sig + a2 * s2 * opf);
    g.Itt = -opf;
    g.Itr = f;
    g.Irr = (r * r - 2.0f * m * r + a2) * iS;
    g.Irp = a * iS;
    g.Ihh = iS;
    g.Ipp = iS * rcpf_fast(s2);
    const float Sig_h = -2.0f * a2 * sc;
    const float f_r = 2.0f * m * (a2 * c * c - r * r) * iS * iS;
    const float f_h = -f * Sig_h * iS;
    const float s2_h = 2.0f * sc;
    dr.tt = f_r;
    dr.tr = f_r;
    dr.tp = -a * s2 * f_r;
    dr.rr = f_r;
    dr.rp = -a * s2 * f_r;
    dr.hh = 2.0f * r;
    dr.pp = s2 * (2.0f * r + a2 * s2 * f_r);
    dh.tt = f_h;
    dh.tr = f_h;
    dh.tp = -a * (f_h * s2 + f * s2_h);
    dh.rr = f_h;
    dh.rp = -a * (s2_h * opf + s2 * f_h);
    dh.hh = Sig_h;
    dh.pp = s2_h * (Sig + a2 * s2 * opf) + s2 * (Sig_h + a2 * (s2_h * opf + s2 * f_h));
}

KRT_HD void lower_f(const MetricF& g, const float v[4], float o[4]) {
    o[0] = g.tt * v[0] + g.tr * v[1] + g.tp * v[3];
    o[1] = g.tr * v[0] + g.rr * v[1] + g.rp * v[3];
    o[2] = g.hh * v[2];
    o[3] = g.tp * v[0] + g.rp * v[1] + g.pp * v[3];
}

KRT_HD void raise_f(const MetricF& g, const float v[4], float o[4]) {
    o[0] = g.Itt * v[0] + g.Itr * v[1];
    o[1] = g.Itr * v[0] + g.Irr * v[1] + g.Irp * v[3];
    o[2] = g.Ihh * v[2];
    o[3] = g.Irp * v[1] + g.Ipp * v[3];
}

KRT_HD float dot_f(const MetricF& g, const float x[4], const float y[4]) {
    float yl[4];
    lower_f(g, y, yl);
    return x[0] * yl[0] + x[1] * yl[1] + x[2] * yl[2] + x[3] * yl[3];
}

// A^mu_b = Gamma^mu_ab K^a (row-major A[mu][b]).
KRT_HD void connection_f(const MetricF& g, const MetricDF& dr, const MetricDF& dh,
                         const float K[4], float A[16]) {
    float vr[4], vh[4];
    vr[0] = dr.tt * K[0] + dr.tr * K[1] + dr.tp * K[3];
    vr[1] = dr.tr * K[0] + dr.rr * K[1] + dr.rp * K[3];
    vr[2] = dr.hh * K[2];
    vr[3] = dr.tp * K[0] + dr.rp * K[1] + dr.pp * K[3];
    vh[0] = dh.tt * K[0] + dh.tr * K[1] + dh.tp * K[3];
    vh[1] = dh.tr * K[0] + dh.rr * K[1] + dh.rp * K[3];
    vh[2] = dh.hh * K[2];
    vh[3] = dh.tp * K[0] + dh.rp * K[1] + dh.pp * K[3];
    const float kr = K[1], kh = K[2];
    const float Mtt = kr * dr.tt + kh * dh.tt, Mtr = kr * dr.tr + kh * dh.tr;
    const float Mtp = kr * dr.tp + kh * dh.tp, Mrr = kr * dr.rr + kh * dh.rr;
    const float Mrp = kr * dr.rp + kh * dh.rp, Mhh = kr * dr.hh + kh * dh.hh;
    const float Mpp = kr * dr.pp + kh * dh.pp;
    // T_{nu b} entry by entry over the non-zero terms (as the FP64 connection)
    const float Ttt = Mtt, Ttr = Mtr + vr[0], Tth = vh[0], Ttp = Mtp;
    const float Trt = Mtr - vr[0], Trr = Mrr, Trh = vh[1] - vr[2], Trp = Mrp - vr[3];
    const float Tht = -vh[0], Thr = vr[2] - vh[1], Thh = Mhh, Thp = -vh[3];
    const float Tpt = Mtp, Tpr = Mrp + vr[3], Tph = vh[3], Tpp = Mpp;
    const float htt = 0.5f * g.Itt, htr = 0.5f * g.Itr, hrr = 0.5f * g.Irr, hrp = 0.5f * g.Irp;
    const float hhh = 0.5f * g.Ihh, hpp = 0.5f * g.Ipp;
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

struct PlasmaF {
    float ne, thetae, B;
    float u[4], b[4];
};

// Analytic ADAF (same model as the FP64 path).
KRT_HD bool adaf_plasma_f(const F32Consts& C, float r, const MetricF& g, PlasmaF& p) {
    const float sr = sqrtf_fast(r);
    p.ne = C.n0 * rcpf_fast(r * sr) * expf_fast(-g.c * g.c * C.ih2);
    const float ir = rcpf_fast(r);
    p.thetae = C.thr * ir;
    p.B = sqrtf_fast(C.cB2 * p.ne * ir);
    float Om = 0.0f, norm = 1.0f;
    const bool kepler = (C.m != 0.0f) && (r >= C.risco);
    if (kepler) {
        Om = rcpf_fast(r * sr + C.a);
        norm = g.tt + 2.0f * g.tp * Om + g.pp * Om * Om;
    }
    if (!kepler || !(norm < 0.0f)) {
        Om = -g.tp * rcpf_fast(g.pp);
        norm = g.tt + 2.0f * g.tp * Om + g.pp * Om * Om;
    }
    if (!(norm < 0.0f)) return false;
    const float ut = rsqrtf_fast(-norm);
    p.u[0] = ut;
    p.u[1] = 0.0f;
    p.u[2] = 0.0f;
    p.u[3] = Om * ut;
    const float uph = g.tp * ut + g.pp * p.u[3];
    const float sc = p.B * rsqrtf_fast(g.pp + uph * uph);
    p.b[0] = sc * uph * p.u[0];
    p.b[1] = 0.0f;
    p.b[2] = 0.0f;
    p.b[3] = sc * (1.0f + uph * p.u[3]);
    return true;
}

// Gridded snapshot: same grid, inversion, interpolation and closure as the
// FP64 path, in FP32 (primitives FP64 or FP32).  The x3 grid coordinate X2
// arrives already reduced to [0, n3) in FP64.
template <class P>
KRT_HD void snapshot_interp_f(const P* prims, int n1, int n2, int n3, float X0, float X1, float X2,
                              float out[8]) {
    int i0[3], i1[3];
    float d[3];
    const float Xv[2] = {X0, X1};
    const int nn[2] = {n1, n2};
    for (int k = 0; k < 2; ++k) {
        const float f = floorf(Xv[k]);
        int i = (int)f;
        float t = Xv[k] - f;
        if (i < 0) { i = 0; t = 0.0f; }
        if (i > nn[k] - 2) { i = nn[k] - 2; t = 1.0f; }
        i0[k] = i;
        i1[k] = i + 1;
        d[k] = t;
    }
    {
        const float f = floorf(X2);
        int i = (int)f;
        // X2 lies in [0, n3] up to the reduction's rounding: one period
        // corrects the index
        i = i < 0 ? i + n3 : (i >= n3 ? i - n3 : i);
        i0[2] = i;
        i1[2] = i + 1 == n3 ? 0 : i + 1;
        d[2] = X2 - f;
    }
    for (int q = 0; q < 8; ++q) out[q] = 0.0f;
    for (int c = 0; c < 8; ++c) {
        const int ia = (c & 4) ? i1[0] : i0[0];
        const int ib = (c & 2) ? i1[1] : i0[1];
        const int ic = (c & 1) ? i1[2] : i0[2];
        const float w = ((c & 4) ? d[0] : 1.0f - d[0]) * ((c & 2) ? d[1] : 1.0f - d[1]) *
                        ((c & 1) ? d[2] : 1.0f - d[2]);
        const P* cell = prims + 8 * (((size_t)ia * n2 + ib) * n3 + ic);
        for (int q = 0; q < 8; ++q) out[q] += w * (float)cell[q];
    }
}

// Returns 1, or 2 when the gathered primitives are not finite (in FP32:
// values beyond its range count as non-finite).
template <class P>
KRT_HD int snapshot_plasma_f(const F32Consts& C, const P* prims, int n1, int n2, int n3, float r,
                             float th, float X2, const MetricF& g, PlasmaF& p) {
    const float x1 = logf_fast(r);
    const float kPif = 3.14159265f;
    // (Newton from theta / pi: with the hardware sine and cosine an iteration
    // costs about what the FP64 path's start table would)
    float x2 = th * (1.0f / kPif);
    float cs2 = 1.0f;
    for (int it = 0; it < 8; ++it) {
        float sn;
        sincos_turns_f(x2, sn, cs2);
        const float dx = (kPif * x2 + C.hh * sn - th) * rcpf_fast(kPif * (1.0f + 2.0f * C.hh * cs2));
        x2 -= dx;
        if (fabsf(dx) < 1e-7f) break;
    }
    {
        float sn;
        sincos_turns_f(x2, sn, cs2);
    }
    float Pv[8];
    snapshot_interp_f(prims, n1, n2, n3, (x1 - C.x1s) * C.idx1 - 0.5f, (x2 - C.x2s) * C.idx2 - 0.5f,
                      X2, Pv);
    if (!(fabsf(Pv[0] + Pv[1] + Pv[2] + Pv[3] + Pv[4] + Pv[5] + Pv[6] + Pv[7]) <= 3.4028235e38f)) return 2;
    const float rho = Pv[0], uu = Pv[1];
    const float J2 = kPif * (1.0f + 2.0f * C.hh * cs2);
    const float U1 = Pv[2] * r, U2 = Pv[3] * J2, U3 = Pv[4];
    const float B1 = Pv[5] * r, B2 = Pv[6] * J2, B3 = Pv[7];
    const float q = g.rr * U1 * U1 + 2.0f * g.rp * U1 * U3 + g.hh * U2 * U2 + g.pp * U3 * U3;
    const float gamma = sqrtf_fast(1.0f + q);
    const float lapse = rsqrtf_fast(-g.Itt);
    p.u[0] = gamma * sqrtf_fast(-g.Itt);   // gamma / lapse
    p.u[1] = U1 - gamma * lapse * g.Itr;
    p.u[2] = U2;
    p.u[3] = U3;
    float ul[4];
    lower_f(g, p.u, ul);
    const float bt = B1 * ul[1] + B2 * ul[2] + B3 * ul[3];
    const float iut = rcpf_fast(p.u[0]);
    p.b[0] = bt;
    p.b[1] = (B1 + bt * p.u[1]) * iut;
    p.b[2] = (B2 + bt * p.u[2]) * iut;
    p.b[3] = (B3 + bt * p.u[3]) * iut;
    const float bsq = dot_f(g, p.b, p.b);
    p.B = sqrtf_fast(bsq > 0.0f ? bsq : 0.0f) * C.B_unit;
    p.ne = rho * C.ne_unit;
    float thetae = 0.0f;
    if (rho > 0.0f && uu > 0.0f) {
        const float ib = 0.5f * bsq * rcpf_fast(C.gm1 * uu);
        const float ib2 = ib * ib;
        const float trat = (C.Rhigh + C.Rlow * ib2) * rcpf_fast(1.0f + ib2);
        thetae = C.mpme * C.gm1 * uu * rcpf_fast(rho * (1.0f + trat));
    }
    p.thetae = thetae;
    if (!(rho > 0.0f) || bsq > C.sigma_cut * rho || r > C.rmax) p.ne = 0.0f;
    return 1;
}

// K0/K2 and K1/K2 of x = 1/Theta_e from the FP32 copy of the Chebyshev table
// (same panels as the FP64 path).
KRT_HD void bessel_ratios_f(const float* __restrict__ tab, float x, float& k0k2, float& k1k2) {
    if (x > 700.0f) {
        // leading terms of the asymptotic series: K0/K2 ~ (1 - 1/(8x)) / (1 + 15/(8x)),
        // K1/K2 ~ (1 + 3/(8x)) / (1 + 15/(8x)), with the next order included
        const float ix = rcpf_fast(x);
        const float s0 = 1.0f - 0.125f * ix + 0.0703125f * ix * ix;
        const float s1 = 1.0f + 0.375f * ix - 0.1171875f * ix * ix;
        const float s2 = 1.0f + 1.875f * ix + 0.8203125f * ix * ix;
        const float is2 = rcpf_fast(s2);
        k0k2 = s0 * is2;
        k1k2 = s1 * is2;
        return;
    }
    if (x < 1e-8f) {
        k0k2 = 0.5f * x * x * (-logf(0.5f * x) - 0.5772157f);
        k1k2 = 0.5f * x;
        return;
    }
    // panel and Chebyshev variable from the bits of x (as bessel_panel)
    const int bits = __float_as_int(x);
    const int e = ((bits >> 23) & 0xff) - 127;
    const int k = (bits >> 21) & (kBesSub - 1);
    const float m = __int_as_float((bits & 0x007fffff) | 0x3f800000);
    const float z = 8.0f * m - (float)(9 + 2 * k);
    int pn = (e - kBesE0) * kBesSub + k;
    pn = pn < 0 ? 0 : (pn >= kBesPanels ? kBesPanels - 1 : pn);
    const float* c0 = tab + pn * 2 * kBesCoef;
    const float* c1 = c0 + kBesCoef;
    float b = c0[kBesDeg], d = c1[kBesDeg];
    for (int kk = kBesDeg - 1; kk >= 0; --kk) {
        b = fmaf(b, z, c0[kk]);
        d = fmaf(d, z, c1[kk]);
    }
    k0k2 = b;
    k1k2 = d;
}

// Thermal coefficients in FP32 at redshift factor g = nu / nu_cam.  Writes
// (a_I, a_Q, a_V, r_Q, r_V) in cm^-1 and returns the scaled source function
// 2^160 B_nu / nu^3 where a_I > 0 (else 0).
KRT_HD float thermal_f(const F32Consts& C, const float* __restrict__ tab, float ne, float thetae,
                       float B, float gz, float cth, float out[5]) {
    for (int k = 0; k < 5; ++k) out[k] = 0.0f;
    if (!(ne > 0.0f) || !(thetae > 0.0f) || !(B > 0.0f) || !(gz > 0.0f)) return 0.0f;
    cth = cth > 1.0f ? 1.0f : (cth < -1.0f ? -1.0f : cth);
    const float sth = sqrtf_fast(1.0f - cth * cth);
    const float nuB = (float)kNuBPerB * B;
    const float iTh = rcpf_fast(thetae);
    float k0k2, k1k2;
    bessel_ratios_f(tab, iTh, k0k2, k1k2);
    const float ig = rcpf_fast(gz);
    const float ig2 = ig * ig;
    out[4] = C.cRV * ne * nuB * cth * ig2 * k0k2;
    if (sth < 1e-10f) return 0.0f;
    out[3] = C.cRQ * ne * nuB * nuB * sth * sth * ig2 * ig * (k1k2 + 6.0f * thetae);
    const float nuc = 1.5f * nuB * sth * thetae * thetae;
    // x^(-1/3) and x^(1/3) = x x^(-2/3), x = nu / nu_c
    // (capped at 1e30, where the emission is zero already: keeps the cube root finite)
    const float xx = fminf(C.nu_cam * gz * rcpf_fast(nuc), 1e30f);
    const float xm13 = rcbrtf_fast(xx);
    const float xm23 = xm13 * xm13;
    const float x13 = xx * xm23;
    const float ex = expf_fast(-1.8899f * x13);
    const float II = 2.5651f * (1.0f + 1.92f * xm13 + 0.9977f * xm23) * ex;
    const float IQ = 2.5651f * (1.0f + 0.93193f * xm13 + 0.499873f * xm23) * ex;
    const float IV = (1.81348f * xm23 * xm13 + 3.42319f * xm23 + 0.0292545f * xm13 * sqrtf_fast(xm13) +
                      2.03773f * xm13) * ex;
    const float pre = C.cJ * ne * gz * iTh * iTh;
    const float jI = pre * II;
    float jQ = pre * IQ;
    float jV = pre * (4.0f / 3.0f) * (cth * rcpf_fast(sth)) * iTh * IV;
    const float jP = hypotf(jQ, jV);
    if (jP > jI) {
        const float sc = jI / jP;
        jQ *= sc;
        jV *= sc;
    }
    const float em1 = expm1f_fast(C.cHnu * gz * iTh);
    const float iem1 = rcpf_fast(em1);
    const float Bnu = C.cBnu * gz * gz * gz * iem1;
    if (jI > 0.0f && Bnu > 0.0f) {
        const float iB = rcpf_fast(Bnu);
        out[0] = jI * iB;
        out[1] = jQ * iB;
        out[2] = jV * iB;
        return out[0] > 0.0f ? C.cSeq * iem1 : 0.0f;
    }
    return 0.0f;
}

// Fluid tetrad legs (same construction as the FP64 path).
KRT_HD float det3_f(float a0, float a1, float a2, float b0, float b1, float b2, float c0, float c1,
                    float c2) {
    return a0 * (b1 * c2 - b2 * c1) - a1 * (b0 * c2 - b2 * c0) + a2 * (b0 * c1 - b1 * c0);
}

KRT_HD void fluid_legs_f(const MetricF& g, const float u[4], const float K[4], const float b[4],
                         float Ku, float e1[4], float l1[4], float e2[4], float l2[4]) {
    float e3[4], l3[4], ul[4];
    for (int k = 0; k < 4; ++k) e3[k] = K[k] + Ku * u[k];
    lower_f(g, e3, l3);
    const float i3 = rsqrtf_fast(e3[0] * l3[0] + e3[1] * l3[1] + e3[2] * l3[2] + e3[3] * l3[3]);
    for (int k = 0; k < 4; ++k) {
        e3[k] *= i3;
        l3[k] *= i3;
    }
    lower_f(g, u, ul);
    float v[4];
    {
        const float bu = b[0] * ul[0] + b[1] * ul[1] + b[2] * ul[2] + b[3] * ul[3];
        const float b3 = b[0] * l3[0] + b[1] * l3[1] + b[2] * l3[2] + b[3] * l3[3];
        for (int k = 0; k < 4; ++k) v[k] = b[k] + bu * u[k] - b3 * e3[k];
    }
    const float bb = dot_f(g, b, b);
    float vv = dot_f(g, v, v);
    if (!(bb > 0.0f) || !(vv >= 1e-12f * bb)) {
        for (int c = 0; c < 2; ++c) {
            const int dir = (c == 0) ? 2 : 1;
            const float cn2 = dir == 2 ? g.hh : g.rr;
            const float pu = ul[dir], p3 = l3[dir];
            for (int k = 0; k < 4; ++k) v[k] = ((k == dir) ? 1.0f : 0.0f) + pu * u[k] - p3 * e3[k];
            vv = dot_f(g, v, v);
            if (vv >= 1e-12f * cn2) break;
        }
    }
    const float iv = rsqrtf_fast(vv);
    for (int k = 0; k < 4; ++k) e2[k] = v[k] * iv;
    lower_f(g, e2, l2);
    const float sg = g.Sig * g.s;
    const float* P = u;
    const float* Q = e2;
    const float* R = e3;
    l1[0] = -sg * det3_f(P[1], P[2], P[3], Q[1], Q[2], Q[3], R[1], R[2], R[3]);
    l1[1] = sg * det3_f(P[0], P[2], P[3], Q[0], Q[2], Q[3], R[0], R[2], R[3]);
    l1[2] = -sg * det3_f(P[0], P[1], P[3], Q[0], Q[1], Q[3], R[0], R[1], R[3]);
    l1[3] = sg * det3_f(P[0], P[1], P[2], Q[0], Q[1], Q[2], R[0], R[1], R[2]);
    raise_f(g, l1, e1);
}

KRT_HD void gen_apply_f(float AQ, float AV, float RQ, float RV, const float v[4], float o[4]) {
    o[0] = -(AQ * v[1] + AV * v[3]);
    o[1] = -(AQ * v[0] + RV * v[2]);
    o[2] = -(-RV * v[1] + RQ * v[3]);
    o[3] = -(AV * v[0] - RQ * v[2]);
}

// Increment dS of the exact constant-coefficient update over w (same closed
// form as the FP64 path), for the scaled Stokes vector S and scaled source
// Seq: S' - S = U - (1 - d0) D with D = S - Seq e0 and
// U = G (d1 D + G (d2 D + G d3 D)).  The generator enters pre-multiplied by w.
KRT_HD void mueller_delta_f(float Seq, float tau, float AQ, float AV, float RQ, float RV,
                            const float S[4], float dS[4]) {
    const float D[4] = {S[0] - Seq, S[1], S[2], S[3]};
    if (tau > 1e15f) {  // fully thermalised over the step
        for (int k = 0; k < 4; ++k) dS[k] = -D[k];
        return;
    }
    // invariants, computed on the generator scaled by sc so that they stay in range
    const float sc = fmaxf(1.0f, fmaxf(tau, fabsf(RQ) + fabsf(RV)));
    const float isc = rcpf_fast(sc);
    const float aq = AQ * isc, av = AV * isc, rq = RQ * isc, rv = RV * isc;
    const float a2 = aq * aq + av * av, r2 = rq * rq + rv * rv, ar = aq * rq + av * rv;
    const float q = 0.5f * (a2 - r2);
    const float rad = sqrtf_fast(q * q + ar * ar);
    float Xs, Ys;
    if (q >= 0.0f) {
        Xs = rad + q;
        // Y = ar^2 / X <= |ar| <= X: below 1e-30 it is dropped (the hardware
        // reciprocal does not take subnormal inputs)
        Ys = (Xs > 1e-30f) ? ar * ar * rcpf_fast(Xs) : 0.0f;
    } else {
        Ys = rad - q;
        Xs = (Ys > 1e-30f) ? ar * ar * rcpf_fast(Ys) : 0.0f;
    }
    const float X = Xs * sc * sc, Y = Ys * sc * sc;
    const float XY = X + Y;
    float omd0, d1, d2, d3;
    if (XY < 0.1f) {
        const float et = expf_fast(-tau);
        const float Z = -Y;
        float h = 1.0f, zk = 1.0f;
        float c2 = 0.0f, c3 = 0.0f, s0 = 0.0f, s1 = 0.0f;
#pragma unroll
        for (int k = 1; k <= 5; ++k) {
            c2 += h * (float)kInvFact[2 * k];
            c3 += h * (float)kInvFact[2 * k + 1];
            s0 += h * (float)kInvFact[2 * k + 2];
            s1 += h * (float)kInvFact[2 * k + 3];
            zk *= Z;
            h = X * h + zk;
        }
        const float XZ = X * Z;
        omd0 = -expm1f_fast(-tau) + et * XZ * s0;
        d1 = et * (1.0f - XZ * s1);
        d2 = et * c2;
        d3 = et * c3;
    } else {
        const float x = sqrtf_fast(X), y = sqrtf_fast(Y);
        const float u = expf_fast(0.5f * (x - tau)), v = expf_fast(-0.5f * (x + tau));
        const float ep = u * u, em = v * v, et = u * v;
        const float ch = 0.5f * (ep + em);
        const float shx = (x > 1e-4f) ? 0.5f * (ep - em) * rcpf_fast(x) : et;
        float sy, cy;
        sincosf(y, &sy, &cy);
        const float syy = (y > 1e-4f) ? sy * rcpf_fast(y) : 1.0f;
        const float iXY = rcpf_fast(XY);
        d1 = (Y * shx + X * et * syy) * iXY;
        d2 = (ch - et * cy) * iXY;
        d3 = (shx - et * syy) * iXY;
        const float qh = 0.5f * (u - v);
        const float s2h = (cy > 0.0f) ? sy * sy * rcpf_fast(2.0f * (1.0f + cy)) : 0.5f * (1.0f - cy);
        omd0 = -expm1f_fast(-tau) + 2.0f * (X * et * s2h - Y * qh * qh) * iXY;
    }
    float T[4], U[4];
    for (int k = 0; k < 4; ++k) T[k] = d3 * D[k];
    gen_apply_f(AQ, AV, RQ, RV, T, U);
    for (int k = 0; k < 4; ++k) T[k] = d2 * D[k] + U[k];
    gen_apply_f(AQ, AV, RQ, RV, T, U);
    for (int k = 0; k < 4; ++k) T[k] = d1 * D[k] + U[k];
    gen_apply_f(AQ, AV, RQ, RV, T, U);
    for (int k = 0; k < 4; ++k) dS[k] = U[k] - omd0 * D[k];
}

// Coherency matrix in FP32 (packed as the FP64 Coh).
struct CohF {
    float R[10];
    float I[6];
};

KRT_HD float nrf(const CohF& N, int i, int j) { return N.R[sym_idx(i, j)]; }
KRT_HD float nif(const CohF& N, int i, int j) {
    return (i == j) ? 0.0f : ((i < j) ? N.I[asym_idx(i, j)] : -N.I[asym_idx(j, i)]);
}

KRT_HD void to_scaled_f(const Coh& N, CohF& F) {
#pragma unroll
    for (int k = 0; k < 10; ++k) F.R[k] = (float)(N.R[k] * kIScale);
#pragma unroll
    for (int k = 0; k < 6; ++k) F.I[k] = (float)(N.I[k] * kIScale);
}

// dN/dlam = -(A N + N A^T) for the scaled FP32 matrix, entry by entry as one
// fused multiply-add chain over the non-zero terms (as transport_rhs).
KRT_HD void transport_rhs_f(const float A[16], const CohF& N, CohF& F) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = i; j < 4; ++j) {
            float s = A[i * 4] * nrf(N, 0, j);
            s = fmaf(nrf(N, i, 0), A[j * 4], s);
#pragma unroll
            for (int b = 1; b < 4; ++b) {
                s = fmaf(A[i * 4 + b], nrf(N, b, j), s);
                s = fmaf(nrf(N, i, b), A[j * 4 + b], s);
            }
            F.R[sym_idx(i, j)] = -s;
        }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = i + 1; j < 4; ++j) {
            float s = A[i * 4] * nif(N, 0, j);
#pragma unroll
            for (int b = 1; b < 4; ++b)
                if (b != j) s = fmaf(A[i * 4 + b], nif(N, b, j), s);
#pragma unroll
            for (int b = 0; b < 4; ++b)
                if (b != i) s = fmaf(nif(N, i, b), A[j * 4 + b], s);
            F.I[asym_idx(i, j)] = -s;
        }
}

KRT_HD void coh_project_f(const CohF& N, const float l1[4], const float l2[4], float S[4]) {
    float n11 = 0.0f, n22 = 0.0f, n12 = 0.0f, m12 = 0.0f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        float y1 = 0.0f, y2 = 0.0f, z2 = 0.0f;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            y1 += nrf(N, i, j) * l1[j];
            y2 += nrf(N, i, j) * l2[j];
            if (j != i) z2 += nif(N, i, j) * l2[j];
        }
        n11 += l1[i] * y1;
        n12 += l1[i] * y2;
        n22 += l2[i] * y2;
        m12 += l1[i] * z2;
    }
    S[0] = n11 + n22;
    S[1] = n11 - n22;
    S[2] = 2.0f * n12;
    S[3] = -2.0f * m12;
}

// N += (coherency matrix of the Stokes increment dS on legs e1, e2) / 2^160,
// formed in FP32 and added in FP64.
// (dN^ij = e1^i p^j + e2^i q^j with p = n11 e1 + nre e2, q = n22 e2 + nre e1,
// as coh_rebuild.)
KRT_HD void coh_add_delta_f(Coh& N, const float dS[4], const float e1[4], const float e2[4]) {
    const float n11 = 0.5f * (dS[0] + dS[1]), n22 = 0.5f * (dS[0] - dS[1]);
    const float nre = 0.5f * dS[2], nim = -0.5f * dS[3];
    float p[4], q[4], r1[4], r2[4];
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
        for (int j = i; j < 4; ++j)
            N.R[sym_idx(i, j)] += kIScaleInv * (double)(e1[i] * p[j] + e2[i] * q[j]);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = i + 1; j < 4; ++j)
            N.I[asym_idx(i, j)] += kIScaleInv * (double)(e1[i] * r2[j] - e2[i] * r1[j]);
}

}  // namespace krt
