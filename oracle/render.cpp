/*
 * Whole-image driver and image reduction.  Test infrastructure only (CPU
 * oracle).
 *
 * Sec. 2.1: one ray per camera pixel, rays independent, parallelised with
 * OpenMP threads; the product is one fully polarized image (Table 1 caption:
 * Stokes I, Q, U, V).  Per pixel: camera launch, backward geodesic saved in
 * full, forward transfer along it.  A ray whose last point is non-finite, or
 * lies on the polar axis (sin(theta) < 1e-12, where the spherical coordinate
 * frame is singular), is transferred over the points before that one; a pixel whose Stokes vector comes out non-finite is
 * written as zeros with status NONFINITE.
 *
 * Reduction: F_S = 1e23 dOmega sum S_ij (Jy), dOmega = (fov_x L/(nx D))
 * (fov_y L/(ny D)), Neumaier-compensated sum in row-major order.
 */
#include <cmath>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif
#include "oracle_internal.h"

extern "C" {

int or_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

int or_render(const or_camera* cam, const or_units* units, const or_model* model,
              const or_snapshot* snap, int64_t npix, const int64_t* pix, double* stokes,
              uint8_t* status, int32_t* nsteps, int32_t nthreads) {
    using namespace orc;
    if (validate_camera(cam) != 0 || validate_model(model, snap, cam) != 0) return -1;
    if (!units || !(units->M_bh_g > 0.0) || !(units->dist_cm > 0.0)) return -1;
    int64_t total = (int64_t)cam->nx * cam->ny;
    if (!pix) npix = total;
    if (npix < 0) return -1;
    if (pix)
        for (int64_t k = 0; k < npix; ++k)
            if (pix[k] < 0 || pix[k] >= total) return -1;
    CameraFrame cf;
    camera_frame(cam, &cf);
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
#endif
    for (int64_t k = 0; k < npix; ++k) {
        int64_t p = pix ? pix[k] : k;
        int32_t i = (int32_t)(p % cam->nx), j = (int32_t)(p / cam->nx);
        double alpha, beta;
        pixel_position(cam, i, j, &alpha, &beta);
        double X[4], K[4];
        launch(cam, cf, alpha, beta, X, K);
        std::vector<double> path;
        int32_t n_end = 0, st = 0;
        trace(cam, X, K, path, cam->max_steps, &n_end, &st);
        /* the stopping point of a non-finite or axis ray lies where the
         * coordinate frame fails: transfer over the points before it */
        int32_t n_use = (st == OR_NONFINITE || st == OR_AXIS) ? n_end - 1 : n_end;
        double ex[4], ey[4], S[4];
        screen_legs(cam, cf, alpha, beta, ex, ey);
        transfer(cam, units, model, snap, ex, ey, path.data(), n_use, S);
        bool ok = std::isfinite(S[0]) && std::isfinite(S[1]) && std::isfinite(S[2]) &&
                  std::isfinite(S[3]);
        if (!ok) {
            S[0] = S[1] = S[2] = S[3] = 0.0;
            st = OR_NONFINITE;
        }
        for (int s = 0; s < 4; ++s) stokes[s * npix + k] = S[s];
        if (status) status[k] = (uint8_t)st;
        if (nsteps) nsteps[k] = n_end;
    }
    return 0;
}

void or_reduce(const or_camera* cam, const or_units* units, const double* stokes,
               double flux_jy[4], double* imax) {
    using namespace orc;
    double L_cm = G_NEWTON * units->M_bh_g / (C_LIGHT * C_LIGHT);
    double dOm = (cam->fov_x * L_cm / (cam->nx * units->dist_cm)) *
                 (cam->fov_y * L_cm / (cam->ny * units->dist_cm));
    int64_t npix = (int64_t)cam->nx * cam->ny;
    for (int s = 0; s < 4; ++s) {
        /* Neumaier compensated summation */
        double sum = 0.0, comp = 0.0;
        for (int64_t k = 0; k < npix; ++k) {
            double x = stokes[s * npix + k];
            double t = sum + x;
            if (std::fabs(sum) >= std::fabs(x)) comp += (sum - t) + x;
            else comp += (x - t) + sum;
            sum = t;
        }
        flux_jy[s] = 1e23 * dOm * (sum + comp);
    }
    double mx = -INFINITY;
    for (int64_t k = 0; k < npix; ++k) mx = std::fmax(mx, stokes[k]);
    *imax = mx;
}

void or_metric(double a, double m, double r, double th, double g[16]) {
    orc::Mat4 G;
    orc::metric(a, m, r, th, G);
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) g[4 * i + j] = G[i][j];
}

void or_metric_inverse(double a, double m, double r, double th, double gi[16]) {
    orc::Mat4 G, Gi;
    orc::metric(a, m, r, th, G);
    orc::invert4(G, Gi);
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) gi[4 * i + j] = Gi[i][j];
}

void or_metric_derivs(double a, double m, double r, double th, double dg[64]) {
    double D[4][4][4];
    orc::metric_derivs(a, m, r, th, D);
    for (int k = 0; k < 4; ++k)
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) dg[16 * k + 4 * i + j] = D[k][i][j];
}

void or_christoffel(double a, double m, double r, double th, double G[64]) {
    double C[4][4][4];
    orc::christoffel(a, m, r, th, C);
    for (int k = 0; k < 4; ++k)
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) G[16 * k + 4 * i + j] = C[k][i][j];
}

double or_horizon(double a, double m) { return orc::horizon(a, m); }
double or_isco(double a) { return orc::isco(a); }

}
