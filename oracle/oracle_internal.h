/*
 * Internal declarations of the CPU oracle (test infrastructure only).
 * Physical constants are CODATA-2018 cgs values; geometry uses G = c = M = 1.
 */
#ifndef KRT_ORACLE_INTERNAL_H
#define KRT_ORACLE_INTERNAL_H

#include <complex>
#include <vector>
#include "oracle.h"

namespace orc {

/* CODATA 2018, cgs (defined here once for the oracle). */
constexpr double C_LIGHT = 2.99792458e10;
constexpr double G_NEWTON = 6.67430e-8;
constexpr double H_PLANCK = 6.62607015e-27;
constexpr double K_BOLTZ = 1.380649e-16;
constexpr double E_CHARGE = 4.803204712570263e-10;
constexpr double M_ELECTRON = 9.1093837015e-28;
constexpr double M_PROTON = 1.67262192369e-24;
constexpr double M_SUN = 1.98841e33;
constexpr double PARSEC = 3.0856775814913673e18;
constexpr double PI = 3.14159265358979323846;

typedef double Mat4[4][4];
typedef std::complex<double> cplx;
typedef cplx CMat4[4][4];

/* kerr.cpp */
void metric(double a, double m, double r, double th, Mat4 g);
void metric_derivs(double a, double m, double r, double th, double dg[4][4][4]);
int invert4(const Mat4 A, Mat4 Ainv);
void christoffel(double a, double m, double r, double th, double G[4][4][4]);
double horizon(double a, double m);
double isco(double a);
double dot(const Mat4 g, const double x[4], const double y[4]);
void lower(const Mat4 g, const double x[4], double xl[4]);

/* camera.cpp */
struct CameraFrame {
    double X[4];
    double e[4][4];   /* e0 (static observer), e_r, e_th, e_ph */
};
int validate_camera(const or_camera* cam);
void camera_frame(const or_camera* cam, CameraFrame* cf);
void launch(const or_camera* cam, const CameraFrame& cf, double alpha, double beta,
            double X[4], double K[4]);
void screen_legs(const or_camera* cam, const CameraFrame& cf, double alpha, double beta,
                 double ex[4], double ey[4]);
void pixel_position(const or_camera* cam, int32_t i, int32_t j, double* alpha, double* beta);

/* geodesic.cpp */
int trace(const or_camera* cam, const double X0[4], const double K0[4],
          std::vector<double>& path, int32_t cap, int32_t* n_end, int32_t* status);

/* plasma.cpp */
struct Plasma {
    double ne, thetae, B;
    double u[4], b[4];
};
int plasma(const or_model* model, const or_snapshot* snap, double a, double m,
           double r, double th, double ph, double L_cm, Plasma* p);
int validate_model(const or_model* model, const or_snapshot* snap, const or_camera* cam);

/* coefficients.cpp */
void bessel_ratios(double x, double* k0k2, double* k1k2);
void kappa_coefficients(int dist, double kappa, double ne, double w, double B, double nu,
                        double cos_thb, double out[8]);
void kappa_integrals(int dist, double kappa, double w, double X, double out[8]);
void thermal_coefficients(double ne, double thetae, double B, double nu, double cos_thb,
                          double out[8]);

/* expm.cpp */
int expm(int n, const double* A, double* E);

/* transfer.cpp */
void mueller_step(const double coef[8], const double S_in[4], double w, double S_out[4]);
int transfer(const or_camera* cam, const or_units* units, const or_model* model,
             const or_snapshot* snap, const double ex[4], const double ey[4],
             const double* path, int32_t n_end, double S_out[4]);

}  // namespace orc

#endif
