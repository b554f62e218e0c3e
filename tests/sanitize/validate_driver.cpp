// Runs the library's host-side parameter checks (krt_validate.hpp, the code
// libkrt.so runs before any launch) on valid inputs and on every kind of
// invalid one, built with AddressSanitizer and UndefinedBehaviorSanitizer
// (tests/test_sanitizers.py).  Exit status 0 when every verdict is the
// expected one and no sanitizer reported.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>

#include "krt_validate.hpp"

static int failures = 0;

static void expect(bool ok, bool want_ok, const char* what) {
    if (ok != want_ok) {
        std::printf("unexpected verdict: %s\n", what);
        ++failures;
    }
}

static krt_camera cam() {
    krt_camera c;
    std::memset(&c, 0, sizeof(c));
    c.struct_size = sizeof(krt_camera);
    c.a = 0.9375;
    c.incl_deg = 60.0;
    c.r_cam = 1000.0;
    c.fov_x = c.fov_y = 40.0;
    c.nx = c.ny = 64;
    c.freq_hz = 230e9;
    c.eps = 0.01;
    c.max_steps = 50000;
    c.jitter = 1;
    c.seed = 1;
    c.mass_factor = 1;
    return c;
}

int main() {
    using namespace krt_host;
    const double nan = std::numeric_limits<double>::quiet_NaN();
    const double inf = std::numeric_limits<double>::infinity();
    expect(check_camera(nullptr).empty(), false, "NULL camera");
    krt_camera c = cam();
    expect(check_camera(&c).empty(), true, "valid camera");
    struct Case { const char* name; void (*edit)(krt_camera&); };
    const Case bad[] = {
        {"struct_size", [](krt_camera& x) { x.struct_size = 3; }},
        {"a = 1", [](krt_camera& x) { x.a = 1.0; }},
        {"a NaN", [](krt_camera& x) { x.a = std::nan(""); }},
        {"r_cam inside", [](krt_camera& x) { x.r_cam = 2.0; }},
        {"r_cam inf", [](krt_camera& x) { x.r_cam = std::numeric_limits<double>::infinity(); }},
        {"nx 0", [](krt_camera& x) { x.nx = 0; }},
        {"ny negative", [](krt_camera& x) { x.ny = -5; }},
        {"huge image", [](krt_camera& x) { x.nx = x.ny = 2147483647; }},
        {"freq 0", [](krt_camera& x) { x.freq_hz = 0.0; }},
        {"eps 0", [](krt_camera& x) { x.eps = 0.0; }},
        {"eps large", [](krt_camera& x) { x.eps = 0.6; }},
        {"max_steps 0", [](krt_camera& x) { x.max_steps = 0; }},
        {"incl 0", [](krt_camera& x) { x.incl_deg = 0.0; }},
        {"incl 180", [](krt_camera& x) { x.incl_deg = 180.0; }},
        {"fov negative", [](krt_camera& x) { x.fov_y = -1.0; }},
        {"mass factor 2", [](krt_camera& x) { x.mass_factor = 2; }},
        {"jitter 3", [](krt_camera& x) { x.jitter = 3; }},
        {"a beyond extremal with m = 0", [](krt_camera& x) { x.mass_factor = 0; x.a = -1.5; }},
    };
    for (const Case& k : bad) {
        krt_camera x = cam();
        k.edit(x);
        expect(check_camera(&x).empty(), false, k.name);
    }
    c.mass_factor = 0;
    c.a = 0.0;
    expect(check_camera(&c).empty(), true, "flat camera");
    for (double a : {-0.999, -0.5, 0.0, 0.3, 0.9375, 0.999}) {
        const double r = isco(a), h = horizon(a, 1.0);
        expect(std::isfinite(r) && r > h && h >= 1.0 && h <= 2.0, true, "isco outside the horizon");
    }

    krt_units u = {sizeof(krt_units), 8.2e39, 2.5e22};
    expect(check_units(&u).empty(), true, "valid units");
    u.dist_cm = -1.0;
    expect(check_units(&u).empty(), false, "negative distance");
    u.dist_cm = inf;
    expect(check_units(&u).empty(), false, "infinite distance");
    expect(check_units(nullptr).empty(), false, "NULL units");

    bool unsup = false;
    krt_adaf ad = {sizeof(krt_adaf), 5e7, 3e11, 10.0, 0.5, 0};
    expect(check_adaf(&ad, &unsup).empty(), true, "valid adaf");
    ad.field_geom = 1;
    expect(check_adaf(&ad, &unsup).empty() || !unsup, false, "unsupported field geometry");
    ad.field_geom = 0;
    ad.beta = nan;
    expect(check_adaf(&ad, &unsup).empty(), false, "NaN beta");

    krt_snapshot_desc d;
    std::memset(&d, 0, sizeof(d));
    d.struct_size = sizeof(d);
    d.n1 = 288;
    d.n2 = 128;
    d.n3 = 128;
    d.dx1 = 0.02;
    d.dx2 = 1.0 / 128;
    d.dx3 = 0.05;
    d.hslope = 0.3;
    d.gamma_ad = 13.0 / 9.0;
    d.M_unit_g = 1e19;
    d.R_high = 40.0;
    d.R_low = 1.0;
    d.sigma_cut = 1.0;
    d.r_emit_max = 50.0;
    int dummy = 0;
    expect(check_snapshot(&d, &dummy, KRT_DTYPE_F64, &unsup).empty(), true, "valid snapshot");
    d.layout = 1;
    expect(check_snapshot(&d, &dummy, KRT_DTYPE_F32, &unsup).empty(), true, "layout 1");
    d.layout = 2;
    expect(check_snapshot(&d, &dummy, KRT_DTYPE_F64, &unsup).empty() || !unsup, false, "layout 2");
    d.layout = 0;
    expect(check_snapshot(&d, &dummy, 7, &unsup).empty() || !unsup, false, "dtype 7");
    expect(check_snapshot(&d, nullptr, KRT_DTYPE_F64, &unsup).empty(), false, "NULL prims");
    d.n1 = d.n2 = d.n3 = 2147483647;
    expect(check_snapshot(&d, &dummy, KRT_DTYPE_F64, &unsup).empty(), false, "huge grid");
    d.n1 = 288;
    d.n2 = 128;
    d.n3 = 128;
    d.hslope = 0.0;
    expect(check_snapshot(&d, &dummy, KRT_DTYPE_F64, &unsup).empty(), false, "hslope 0");

    krt_launch_config lc = {sizeof(krt_launch_config), 8, 0, 0, 1};
    expect(check_launch_config(&lc).empty(), true, "valid launch config");
    lc.tile_w = 12;
    expect(check_launch_config(&lc).empty(), false, "tile_w 12");
    lc.tile_w = 8;
    lc.path_cap = 10;
    expect(check_launch_config(&lc).empty(), false, "path_cap 10");
    if (failures) return 1;
    std::printf("validate driver ok\n");
    return 0;
}
