/*
 * Backward null-geodesic integration with a stored path.
 * Test infrastructure only (CPU oracle).
 *
 * Sec. 2.1: a null geodesic is integrated from the camera for every pixel,
 * backward in time, with an adaptive step controlled by one parameter, and
 * the path is saved.  Sec. 2.2 names that parameter eps.  Readings:
 *  - state y = (X^mu, K^mu), dX/dlam = K, dK^mu/dlam = -Gamma^mu_ab K^a K^b;
 *  - classical fourth-order Runge-Kutta in lam, no error control;
 *  - step |dlam| = eps / (|K^r|/r + |K^theta| max(1, |cot theta|) + |K^phi|)
 *    at the start of the step, dlam < 0: the step bounds the relative change
 *    of r, the change of theta and phi, and the relative change of sin(theta)
 *    (d ln sin(theta) = cot(theta) dtheta), so a ray that passes close to the
 *    polar axis, where the coordinate frame turns quickly, takes steps that
 *    shrink with its distance to the axis;
 *  - after each step, stop on (in this order) a non-finite component,
 *    sin(theta) < 1e-12, r < 1.05 r_+ (flat space: r < 1e-6), r > r_cam while
 *    moving outward, or the step cap;
 *  - stored per point: r, theta, phi, K^t, K^r, K^theta, K^phi and the dlam of
 *    the step that reached the point (0 at the camera).
 */
#include <cmath>
#include "oracle_internal.h"

namespace orc {

static void rhs(double a, double m, const double y[8], double dy[8]) {
    double G[4][4][4];
    christoffel(a, m, y[1], y[2], G);
    const double* K = y + 4;
    for (int mu = 0; mu < 4; ++mu) {
        dy[mu] = K[mu];
        double s = 0.0;
        for (int al = 0; al < 4; ++al)
            for (int be = 0; be < 4; ++be) s += G[mu][al][be] * K[al] * K[be];
        dy[4 + mu] = -s;
    }
}

static void store(std::vector<double>& path, const double y[8], double dlam) {
    path.push_back(y[1]);
    path.push_back(y[2]);
    path.push_back(y[3]);
    path.push_back(y[4]);
    path.push_back(y[5]);
    path.push_back(y[6]);
    path.push_back(y[7]);
    path.push_back(dlam);
}

/* Returns 0, or -2 if more than cap+1 points would be needed. */
int trace(const or_camera* cam, const double X0[4], const double K0[4],
          std::vector<double>& path, int32_t cap, int32_t* n_end, int32_t* status) {
    const double a = cam->a;
    const double m = (double)cam->mass_factor;
    const double r_stop = (cam->mass_factor == 0) ? 1e-6 : 1.05 * horizon(a, m);
    double y[8];
    for (int k = 0; k < 4; ++k) {
        y[k] = X0[k];
        y[4 + k] = K0[k];
    }
    path.clear();
    store(path, y, 0.0);
    int32_t n = 0;
    for (;;) {
        if (n >= cap) {
            *n_end = n;
            *status = OR_STEP_CAP;
            return -2;
        }
        double cot = std::cos(y[2]) / std::sin(y[2]);
        double h = -cam->eps / (std::fabs(y[5]) / y[1] + std::fabs(y[6]) * std::fmax(1.0, std::fabs(cot)) +
                                std::fabs(y[7]));
        double k1[8], k2[8], k3[8], k4[8], yt[8];
        rhs(a, m, y, k1);
        for (int i = 0; i < 8; ++i) yt[i] = y[i] + 0.5 * h * k1[i];
        rhs(a, m, yt, k2);
        for (int i = 0; i < 8; ++i) yt[i] = y[i] + 0.5 * h * k2[i];
        rhs(a, m, yt, k3);
        for (int i = 0; i < 8; ++i) yt[i] = y[i] + h * k3[i];
        rhs(a, m, yt, k4);
        for (int i = 0; i < 8; ++i) y[i] += h / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
        ++n;
        store(path, y, h);

        bool finite = true;
        for (int i = 0; i < 8; ++i) finite = finite && std::isfinite(y[i]);
        int st = -1;
        if (!finite || !std::isfinite(h)) st = OR_NONFINITE;
        else if (std::sin(y[2]) < 1e-12) st = OR_AXIS;
        else if (y[1] < r_stop) st = OR_CAPTURED;
        else if (y[1] > cam->r_cam && y[5] * h > 0.0) st = OR_ESCAPED;
        else if (n >= cam->max_steps) st = OR_STEP_CAP;
        if (st >= 0) {
            *n_end = n;
            *status = st;
            return 0;
        }
    }
}

}  // namespace orc

extern "C" int or_trace_ray(const or_camera* cam, double alpha, double beta, int32_t cap,
                            double* path, int32_t* n_end, int32_t* status) {
    if (orc::validate_camera(cam) != 0 || cap < 1) return -1;
    orc::CameraFrame cf;
    orc::camera_frame(cam, &cf);
    double X[4], K[4];
    orc::launch(cam, cf, alpha, beta, X, K);
    std::vector<double> p;
    int rc = orc::trace(cam, X, K, p, cap, n_end, status);
    size_t npts = p.size() / 8;
    if (path)
        for (size_t k = 0; k < npts * 8; ++k) path[k] = p[k];
    return rc;
}
