// Host-side validation of the C ABI's parameter structs (plain C++, no HIP):
// every check the library makes before any launch.  libkrt.so includes it,
// and so does the sanitizer test driver, which builds it with AddressSanitizer
// and UndefinedBehaviorSanitizer and runs it on valid and invalid inputs.
// Each check returns an empty message when the struct is valid.
#pragma once

#include <cmath>
#include <cstdint>
#include <initializer_list>
#include <string>

#include "krt.h"

namespace krt_host {

inline bool finite_all(std::initializer_list<double> v) {
    for (double x : v)
        if (!std::isfinite(x)) return false;
    return true;
}

// Outer horizon r_+ = m + sqrt(m^2 - a^2) (0 in the flat test mode).
inline double horizon(double a, double m) { return m == 0.0 ? 0.0 : m + std::sqrt(m * m - a * a); }

// r_isco of Kerr (Bardeen, Press & Teukolsky 1972), prograde for a > 0.
inline double isco(double a) {
    const double aa = std::fabs(a);
    const double z1 = 1.0 + std::cbrt(1.0 - aa * aa) * (std::cbrt(1.0 + aa) + std::cbrt(1.0 - aa));
    const double z2 = std::sqrt(3.0 * aa * aa + z1 * z1);
    return 3.0 + z2 - (a >= 0.0 ? 1.0 : -1.0) * std::sqrt((3.0 - z1) * (3.0 + z1 + 2.0 * z2));
}

// Camera and step control (krt.h: krt_camera).
inline std::string check_camera(const krt_camera* c) {
    if (!c) return "camera is NULL";
    if (c->struct_size != sizeof(krt_camera)) return "camera struct_size mismatch";
    if (!finite_all({c->a, c->incl_deg, c->phi_deg, c->r_cam, c->fov_x, c->fov_y, c->freq_hz, c->eps}))
        return "camera has a non-finite field";
    if (!(std::fabs(c->a) < 1.0)) return "spin must satisfy |a| < 1";
    if (c->mass_factor != 0 && c->mass_factor != 1) return "mass_factor must be 0 or 1";
    if (!(c->r_cam > 0.0) || !(c->r_cam > 2.0 * horizon(c->a, c->mass_factor)))
        return "r_cam must exceed twice the horizon radius";
    if (c->nx < 1 || c->ny < 1) return "nx and ny must be >= 1";
    if ((int64_t)c->nx * c->ny > (int64_t)INT32_MAX / 2) return "image too large";
    if (!(c->freq_hz > 0.0)) return "freq_hz must be > 0";
    if (!(c->eps > 0.0 && c->eps <= 0.5)) return "eps must satisfy 0 < eps <= 0.5";
    if (c->max_steps < 1) return "max_steps must be >= 1";
    if (!(c->incl_deg > 0.0 && c->incl_deg < 180.0)) return "incl_deg must be in (0, 180)";
    if (!(c->fov_x > 0.0 && c->fov_y > 0.0)) return "field of view must be > 0";
    if (c->jitter != 0 && c->jitter != 1) return "jitter must be 0 or 1";
    return "";
}

inline std::string check_units(const krt_units* u) {
    if (!u || u->struct_size != sizeof(krt_units)) return "bad units struct";
    if (!(std::isfinite(u->M_bh_g) && u->M_bh_g > 0.0 && std::isfinite(u->dist_cm) && u->dist_cm > 0.0))
        return "units must be finite and > 0";
    return "";
}

// ADAF parameters; *unsupported is set for valid values the library does not
// implement.
inline std::string check_adaf(const krt_adaf* p, bool* unsupported) {
    *unsupported = false;
    if (!p || p->struct_size != sizeof(krt_adaf)) return "bad adaf struct";
    if (!finite_all({p->n0_cgs, p->T0_K, p->beta, p->h_over_r}) || !(p->n0_cgs >= 0.0) || !(p->T0_K > 0.0) ||
        !(p->beta > 0.0) || !(p->h_over_r > 0.0))
        return "ADAF parameters must be finite, n0 >= 0, T0, beta, h > 0";
    if (p->field_geom != 0) {
        *unsupported = true;
        return "only toroidal fields (0) are supported";
    }
    return "";
}

inline std::string check_snapshot(const krt_snapshot_desc* desc, const void* d_prims, int dtype,
                                  bool* unsupported) {
    *unsupported = false;
    if (!desc || desc->struct_size != sizeof(krt_snapshot_desc)) return "bad snapshot struct";
    if (!d_prims) return "d_prims is NULL";
    if (dtype != KRT_DTYPE_F64 && dtype != KRT_DTYPE_F32) {
        *unsupported = true;
        return "dtype must be KRT_DTYPE_F64 or KRT_DTYPE_F32";
    }
    if (desc->layout != 0 && desc->layout != 1) {
        *unsupported = true;
        return "layout must be 0 ([n1][n2][n3][8]) or 1 ([8][n1][n2][n3])";
    }
    const krt_snapshot_desc& d = *desc;
    if (d.n1 < 2 || d.n2 < 2 || d.n3 < 1) return "grid needs n1, n2 >= 2 and n3 >= 1";
    // at most 2^28 cells (8 fields of 2^31 elements), each product bounded
    // before the next multiplication (no int64 overflow for any input)
    const int64_t lim = ((int64_t)1 << 31) / 8;
    if (d.n1 > lim || d.n2 > lim || d.n3 > lim || (int64_t)d.n1 * d.n2 > lim ||
        (int64_t)d.n1 * d.n2 * d.n3 > lim)
        return "grid too large";
    if (!finite_all({d.x1_start, d.dx1, d.x2_start, d.dx2, d.x3_start, d.dx3, d.hslope, d.gamma_ad, d.M_unit_g,
                     d.R_high, d.R_low, d.sigma_cut, d.r_emit_max}))
        return "snapshot description has a non-finite field";
    if (!(d.dx1 > 0.0 && d.dx2 > 0.0 && d.dx3 > 0.0)) return "cell sizes must be > 0";
    if (!(d.M_unit_g > 0.0) || !(d.gamma_ad > 1.0)) return "need M_unit > 0, gamma_ad > 1";
    if (!(d.hslope > 0.0 && d.hslope <= 1.0)) return "hslope must be in (0, 1]";
    return "";
}

inline std::string check_launch_config(const krt_launch_config* cfg) {
    if (!cfg || cfg->struct_size != sizeof(krt_launch_config)) return "bad config struct";
    const int tw = cfg->tile_w;
    if (!(tw == 4 || tw == 8 || tw == 16 || tw == 32 || tw == 64)) return "tile_w must be 4, 8, 16, 32 or 64";
    if (cfg->blocks_per_cu < 0 || cfg->blocks_per_cu > 16) return "blocks_per_cu must be 0..16";
    if (cfg->path_cap != 0 && (cfg->path_cap < 64 || cfg->path_cap > 65536))
        return "path_cap must be 0 or 64..65536";
    if (cfg->order < 0 || cfg->order > 2) return "order must be 0, 1 or 2";
    return "";
}

}  // namespace krt_host
