/*
 * Camera: pixel grid, jitter, static-observer tetrad and photon launch.
 * Test infrastructure only (CPU oracle).
 *
 * Sec. 2.1: photons are launched from the camera, one per pixel, for a chosen
 * field of view and resolution.  Readings (the paper gives no camera model):
 *  - the camera is a static observer at (r_cam, theta_o, phi_o);
 *  - its tetrad is Gram-Schmidt of (u, d_r, d_theta, d_phi) with respect to g;
 *  - pixel (i, j) sits at alpha = fov_x ((i + 1/2 + dx)/nx - 1/2),
 *    beta = fov_y ((j + 1/2 + dy)/ny - 1/2), with jitter d uniform in
 *    [-1/2, 1/2) drawn from the SplitMix64 finalizer of a counter;
 *  - the arriving photon travels along n ~ e_r - (alpha/r_cam) e_phi
 *    + (beta/r_cam) e_theta, and K = e0 + n so that -K.u_cam = 1;
 *  - image axes: +alpha along e_phi, +beta along -e_theta.
 */
#include <cmath>
#include "oracle_internal.h"

namespace orc {

/* SplitMix64 output function (Steele, Lea & Flood 2014): xor-shift 30,
 * multiply, xor-shift 27, multiply, xor-shift 31. */
static uint64_t splitmix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Jitter component c (0: alpha, 1: beta) of pixel (i, j): the k-th output of
 * a SplitMix64 stream seeded with `seed`, k = 2 (j nx + i) + c + 1, mapped to
 * [-1/2, 1/2) with 53 random bits. */
static double jitter(const or_camera* cam, int32_t i, int32_t j, int c) {
    uint64_t k = 2ULL * ((uint64_t)j * (uint64_t)cam->nx + (uint64_t)i) + (uint64_t)c + 1ULL;
    uint64_t z = splitmix64(cam->seed + k * 0x9E3779B97F4A7C15ULL);
    return (double)(z >> 11) * (1.0 / 9007199254740992.0) - 0.5;
}

void pixel_position(const or_camera* cam, int32_t i, int32_t j, double* alpha, double* beta) {
    double dx = 0.0, dy = 0.0;
    if (cam->jitter) {
        dx = jitter(cam, i, j, 0);
        dy = jitter(cam, i, j, 1);
    }
    *alpha = cam->fov_x * ((i + 0.5 + dx) / cam->nx - 0.5);
    *beta = cam->fov_y * ((j + 0.5 + dy) / cam->ny - 0.5);
}

int validate_camera(const or_camera* cam) {
    if (!cam) return -1;
    const double vals[] = {cam->a, cam->incl_deg, cam->phi_deg, cam->r_cam, cam->fov_x,
                           cam->fov_y, cam->freq_hz, cam->eps};
    for (double v : vals)
        if (!std::isfinite(v)) return -1;
    if (!(std::fabs(cam->a) < 1.0)) return -1;
    if (cam->mass_factor != 0 && cam->mass_factor != 1) return -1;
    double rh = horizon(cam->a, (double)cam->mass_factor);
    if (!(cam->r_cam > 2.0 * rh) || !(cam->r_cam > 0.0)) return -1;
    if (cam->nx < 1 || cam->ny < 1) return -1;
    if (!(cam->freq_hz > 0.0)) return -1;
    if (!(cam->eps > 0.0 && cam->eps <= 0.5)) return -1;
    if (cam->max_steps < 1) return -1;
    if (!(cam->incl_deg > 0.0 && cam->incl_deg < 180.0)) return -1;
    if (!(cam->fov_x > 0.0 && cam->fov_y > 0.0)) return -1;
    return 0;
}

/* Static observer u = d_t / sqrt(-g_tt) and Gram-Schmidt of d_r, d_theta,
 * d_phi against it, in that order. */
void camera_frame(const or_camera* cam, CameraFrame* cf) {
    double m = (double)cam->mass_factor;
    double th = cam->incl_deg * PI / 180.0;
    double ph = cam->phi_deg * PI / 180.0;
    cf->X[0] = 0.0;
    cf->X[1] = cam->r_cam;
    cf->X[2] = th;
    cf->X[3] = ph;
    Mat4 g;
    metric(cam->a, m, cam->r_cam, th, g);
    double (*e)[4] = cf->e;
    for (int k = 0; k < 4; ++k)
        for (int mu = 0; mu < 4; ++mu) e[k][mu] = (k == mu) ? 1.0 : 0.0;
    /* e0: normalise the timelike Killing vector. */
    double n0 = std::sqrt(-g[0][0]);
    for (int mu = 0; mu < 4; ++mu) e[0][mu] /= n0;
    for (int k = 1; k < 4; ++k) {
        double v[4];
        for (int mu = 0; mu < 4; ++mu) v[mu] = e[k][mu];
        /* remove the part along e0 (e0.e0 = -1) */
        double p0 = dot(g, v, e[0]);
        for (int mu = 0; mu < 4; ++mu) v[mu] += p0 * e[0][mu];
        /* remove the parts along the earlier spatial legs */
        for (int l = 1; l < k; ++l) {
            double pl = dot(g, v, e[l]);
            for (int mu = 0; mu < 4; ++mu) v[mu] -= pl * e[l][mu];
        }
        double nv = std::sqrt(dot(g, v, v));
        for (int mu = 0; mu < 4; ++mu) e[k][mu] = v[mu] / nv;
    }
}

/* Spatial direction of travel of the arriving photon, in the camera's
 * orthonormal frame (components along e_r, e_theta, e_phi). */
static void arrival_direction(const or_camera* cam, double alpha, double beta, double n[3]) {
    double ra = alpha / cam->r_cam, rb = beta / cam->r_cam;
    double norm = std::sqrt(1.0 + ra * ra + rb * rb);
    n[0] = 1.0 / norm;
    n[1] = rb / norm;
    n[2] = -ra / norm;
}

void launch(const or_camera* cam, const CameraFrame& cf, double alpha, double beta,
            double X[4], double K[4]) {
    double n[3];
    arrival_direction(cam, alpha, beta, n);
    for (int mu = 0; mu < 4; ++mu) {
        X[mu] = cf.X[mu];
        K[mu] = cf.e[0][mu] + n[0] * cf.e[1][mu] + n[1] * cf.e[2][mu] + n[2] * cf.e[3][mu];
    }
}

/* Polarization legs of the pixel's screen: the image axes e_x = e_phi and
 * e_y = -e_theta made transverse to this pixel's arrival direction n:
 * e_x' = normalised (e_x - (e_x.n) n), e_y' = n x e_x', so that (e_x', e_y', n)
 * is right-handed and both legs are orthogonal to the ray (reading: the
 * screen basis of each pixel is transverse to its own ray). */
void screen_legs(const or_camera* cam, const CameraFrame& cf, double alpha, double beta,
                 double ex[4], double ey[4]) {
    double n[3];
    arrival_direction(cam, alpha, beta, n);
    double x[3] = {0.0, 0.0, 1.0};  /* e_phi in (e_r, e_theta, e_phi) */
    double xn = x[0] * n[0] + x[1] * n[1] + x[2] * n[2];
    for (int k = 0; k < 3; ++k) x[k] -= xn * n[k];
    double nx = std::sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    for (int k = 0; k < 3; ++k) x[k] /= nx;
    /* y = n cross x in the right-handed orthonormal triad (e_r, e_theta, e_phi) */
    double y[3] = {n[1] * x[2] - n[2] * x[1], n[2] * x[0] - n[0] * x[2], n[0] * x[1] - n[1] * x[0]};
    for (int mu = 0; mu < 4; ++mu) {
        ex[mu] = x[0] * cf.e[1][mu] + x[1] * cf.e[2][mu] + x[2] * cf.e[3][mu];
        ey[mu] = y[0] * cf.e[1][mu] + y[1] * cf.e[2][mu] + y[2] * cf.e[3][mu];
    }
}

}  // namespace orc

extern "C" {

uint64_t or_splitmix64(uint64_t x) { return orc::splitmix64(x); }

int or_pixel_position(const or_camera* cam, int32_t i, int32_t j, double* alpha, double* beta) {
    if (orc::validate_camera(cam) != 0) return -1;
    if (i < 0 || j < 0 || i >= cam->nx || j >= cam->ny) return -1;
    orc::pixel_position(cam, i, j, alpha, beta);
    return 0;
}

int or_camera_launch(const or_camera* cam, double alpha, double beta, double X[4], double K[4],
                     double tetrad[16]) {
    if (orc::validate_camera(cam) != 0) return -1;
    orc::CameraFrame cf;
    orc::camera_frame(cam, &cf);
    orc::launch(cam, cf, alpha, beta, X, K);
    for (int k = 0; k < 4; ++k)
        for (int mu = 0; mu < 4; ++mu) tetrad[4 * k + mu] = cf.e[k][mu];
    return 0;
}

}
