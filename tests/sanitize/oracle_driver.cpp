// Runs the CPU oracle on small cases of every kind it computes, built with
// AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_sanitizers.py):
// ADAF images (jitter, pixel subset, step cap), a flat-space slab, a small
// snapshot with and without a non-finite cell, coefficients of both electron
// distributions, the matrix exponential and the path-transfer hook.  Any
// sanitizer report aborts with a non-zero exit status.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "oracle.h"

static or_camera camera(int n, double a, double incl, int mass_factor) {
    or_camera c;
    std::memset(&c, 0, sizeof(c));
    c.a = a;
    c.incl_deg = incl;
    c.r_cam = 1000.0;
    c.fov_x = c.fov_y = 30.0;
    c.nx = c.ny = n;
    c.freq_hz = 230e9;
    c.eps = 0.05;
    c.max_steps = 50000;
    c.jitter = 1;
    c.seed = 3;
    c.mass_factor = mass_factor;
    return c;
}

static int render(const or_camera& c, const or_units& u, const or_model& m, const or_snapshot* s,
                  int64_t npix, const int64_t* pix, double* flux) {
    const int64_t n = pix ? npix : (int64_t)c.nx * c.ny;
    std::vector<double> S(4 * n);
    std::vector<uint8_t> st(n);
    std::vector<int32_t> ns(n);
    const int rc = or_render(&c, &u, &m, s, npix, pix, S.data(), st.data(), ns.data(), 2);
    if (rc != 0) return rc;
    double imax = 0.0;
    if (!pix) or_reduce(&c, &u, S.data(), flux, &imax);
    return 0;
}

int main() {
    const or_units u = {4.14e6 * 1.98841e33, 8.127e3 * 3.0856775814913673e18};
    double flux[4] = {0, 0, 0, 0};
    or_model adaf;
    std::memset(&adaf, 0, sizeof(adaf));
    adaf.kind = OR_MODEL_ADAF;
    adaf.n0_cgs = 5e7;
    adaf.T0_K = 3e11;
    adaf.beta = 10.0;
    adaf.h_over_r = 0.5;
    or_camera c = camera(6, 0.9375, 60.0, 1);
    if (render(c, u, adaf, nullptr, 0, nullptr, flux) != 0 || !(flux[0] > 0.0)) return 1;
    const int64_t pix[3] = {0, 17, 35};
    if (render(c, u, adaf, nullptr, 3, pix, flux) != 0) return 2;
    c.max_steps = 5;
    if (render(c, u, adaf, nullptr, 0, nullptr, flux) != 0) return 3;
    // kappa electrons in the ADAF
    c = camera(3, 0.5, 40.0, 1);
    or_model kap = adaf;
    kap.electrons = 1;
    kap.kappa = 4.0;
    if (render(c, u, kap, nullptr, 0, nullptr, flux) != 0) return 4;

    // flat-space slab
    or_model slab;
    std::memset(&slab, 0, sizeof(slab));
    slab.kind = OR_MODEL_SLAB_PLASMA;
    slab.slab_radius = 10.0;
    slab.slab_ne = 1e6;
    slab.slab_thetae = 3.0;
    slab.slab_B = 30.0;
    slab.slab_bdir[0] = 0.3;
    slab.slab_bdir[2] = 1.0;
    or_camera f = camera(3, 0.0, 90.0, 0);
    f.fov_x = f.fov_y = 4.0;
    if (render(f, u, slab, nullptr, 0, nullptr, flux) != 0) return 5;

    // small snapshot: smooth torus-like fields, then one non-finite cell
    const int n1 = 12, n2 = 8, n3 = 6;
    std::vector<double> P((size_t)n1 * n2 * n3 * 8);
    or_snapshot s;
    std::memset(&s, 0, sizeof(s));
    s.n1 = n1;
    s.n2 = n2;
    s.n3 = n3;
    s.x1_start = std::log(1.2);
    s.dx1 = (std::log(200.0) - std::log(1.2)) / n1;
    s.dx2 = 1.0 / n2;
    s.dx3 = 2.0 * 3.141592653589793 / n3;
    s.hslope = 0.3;
    s.gamma_ad = 13.0 / 9.0;
    s.M_unit_g = 1e19;
    s.R_high = 40.0;
    s.R_low = 1.0;
    s.sigma_cut = 1.0;
    s.r_emit_max = 50.0;
    for (int i = 0; i < n1; ++i)
        for (int j = 0; j < n2; ++j)
            for (int k = 0; k < n3; ++k) {
                double* p = &P[(((size_t)i * n2 + j) * n3 + k) * 8];
                const double r = std::exp(s.x1_start + (i + 0.5) * s.dx1);
                const double x2 = (j + 0.5) * s.dx2;
                p[0] = 30.0 * std::exp(-(r - 15.0) * (r - 15.0) / 72.0 - (x2 - 0.5) * (x2 - 0.5) / 0.02) + 1e-3;
                p[1] = 0.2 * p[0] / r;
                p[4] = 1.0 / (std::pow(r, 1.5) + 0.9);
                p[5] = 0.01 / (r * r);
                p[7] = 0.05 * std::sqrt(p[1]) / r;
            }
    s.prims = P.data();
    or_model snapm;
    std::memset(&snapm, 0, sizeof(snapm));
    snapm.kind = OR_MODEL_SNAPSHOT;
    or_camera cs = camera(5, 0.9, 25.0, 1);
    cs.jitter = 0;
    if (render(cs, u, snapm, &s, 0, nullptr, flux) != 0) return 6;
    P[(((size_t)5 * n2 + 4) * n3 + 2) * 8 + 2] = std::nan("");
    if (render(cs, u, snapm, &s, 0, nullptr, flux) != 0) return 7;

    // coefficients, integrals, matrix exponential, transfer hook
    double co[8];
    or_thermal_coefficients(1e6, 20.0, 10.0, 230e9, 0.4, co);
    or_thermal_coefficients(1e6, 1e-9, 10.0, 230e9, 1.0, co);
    or_kappa_coefficients(OR_DIST_KAPPA, 3.5, 1e6, 5.0, 10.0, 230e9, -0.3, co);
    const double in[6] = {4.0, 3.0, 20.0, 7.5, 60.0, 0.05};
    double out[16];
    or_kappa_integrals(OR_DIST_KAPPA, 2, in, out, 2);
    double A[25], E[25];
    for (int k = 0; k < 25; ++k) A[k] = 0.1 * std::sin(1.0 + k);
    if (or_expm(5, A, E) != 0) return 8;
    const double coef[8] = {1e-3, 2e-4, 1e-4, 0.5, 0.1, 0.05, 2.0, 3.0};
    const double S0[4] = {1.0, 0.2, -0.1, 0.05};
    double S1[4];
    or_mueller_step(coef, S0, 0.3, S1);
    double path[8 * 40];
    int32_t n_end = 0, status = 0;
    c = camera(1, 0.9375, 60.0, 1);
    const int trc = or_trace_ray(&c, 3.0, 2.0, 39, path, &n_end, &status);
    if (trc != -2 && trc != 0) return 9;
    double St[4];
    if (or_transfer_path(&c, &u, &adaf, nullptr, 3.0, 2.0, path, n_end, St) != 0) return 10;
    std::printf("oracle driver ok: flux %.6e\n", flux[0]);
    return 0;
}
