/*
 * Plain FP64 CPU oracle of the polarized Kerr ray tracer.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this library: only the tests, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code, header, table or constant
 * with the GPU library.
 *
 * What it computes (Sec. 2.1 of Moscibrodzka & Yfantis 2023): for every
 * camera pixel, a null geodesic integrated backward in time from the camera
 * with an adaptive step controlled by a parameter eps, saved; then the
 * covariant, fully polarized transfer equation (coherency matrix in the
 * coordinate frame) integrated forward along the saved path toward the
 * camera, with plasma quantities and synchrotron emission, absorption and
 * Faraday rotation/conversion coefficients evaluated at every stored point.
 *
 * Everything the paper leaves open is fixed by the readings listed in the
 * design notes (integrator, step rule, stop rule, camera, plasma models,
 * coefficient fits, splitting).  Units: G = c = M = 1 for geometry, cgs for
 * radiative quantities.  Coordinates: Kerr-Schild (t, r, theta, phi).
 *
 * Functions return 0 on success and a negative code on invalid input.
 */
#ifndef KRT_ORACLE_H
#define KRT_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Camera and integration parameters (Sec. 2.1: spin, viewing angle,
 * frequency, field of view, resolution, step parameter eps of Sec. 2.2). */
typedef struct {
    double a;          /* dimensionless spin, |a| < 1                          */
    double incl_deg;   /* observer polar angle theta_o, degrees                */
    double phi_deg;    /* observer azimuth phi_o, degrees                      */
    double r_cam;      /* camera radius, units of M                            */
    double fov_x;      /* field of view along alpha, units of M                */
    double fov_y;      /* field of view along beta, units of M                 */
    int32_t nx, ny;    /* pixels                                               */
    double freq_hz;    /* observing frequency nu_obs at the camera             */
    double eps;        /* step parameter                                       */
    int32_t max_steps; /* step cap                                             */
    int32_t jitter;    /* 1: SplitMix64 jitter inside each pixel, 0: centres   */
    uint64_t seed;     /* jitter seed                                          */
    int32_t mass_factor; /* 1: Kerr; 0: flat space (test mode)                 */
} or_camera;

typedef struct {
    double M_bh_g;     /* black-hole mass, g                                   */
    double dist_cm;    /* distance to the source, cm                           */
} or_units;

/* Plasma models. */
enum {
    OR_MODEL_ADAF = 0,        /* analytic ADAF-like flow                       */
    OR_MODEL_SLAB_PLASMA = 1, /* flat-space test: uniform cold/thermal ball    */
    OR_MODEL_SLAB_FIXED = 2,  /* flat-space test: given invariant coefficients */
    OR_MODEL_SNAPSHOT = 3     /* gridded GRMHD-like snapshot                   */
};

typedef struct {
    int32_t kind;
    /* ADAF: n_e = n0 r^-3/2 exp(-z^2/(2 (h r)^2)), T_e = T0/r, beta = p/p_mag */
    double n0_cgs, T0_K, beta, h_over_r;
    /* slab models (flat space, a = 0): ball r < slab_radius, static fluid   */
    double slab_radius;
    double slab_ne, slab_thetae, slab_B;  /* cgs, dimensionless, Gauss        */
    double slab_bdir[3];                  /* field direction, Cartesian        */
    double slab_jextra[3];                /* extra invariant emissivity I,Q,V  */
    double slab_coef[8];  /* fixed: J_I J_Q J_V A_I A_Q A_V R_Q R_V (invariant) */
    /* electrons of the ADAF / snapshot models: 0 thermal, 1 kappa of index
     * `kappa` with width Theta_e (the nonthermal module) */
    int32_t electrons;
    double kappa;
    /* 1: the radiative update also at points where every coefficient is zero
     * (projection on the fluid legs and rebuild, as the update is first
     * stated); 0 (the reading both sides use): such points leave N as it is */
    int32_t update_empty;
} or_model;

/* Gridded snapshot description (modified Kerr-Schild grid). */
typedef struct {
    int32_t n1, n2, n3;
    double x1_start, dx1, x2_start, dx2, x3_start, dx3;
    double hslope;
    double gamma_ad;
    double M_unit_g;
    double R_high, R_low;
    double sigma_cut;
    double r_emit_max;
    const double* prims;  /* [n1][n2][n3][8]: rho, u, U1, U2, U3, B1, B2, B3 */
} or_snapshot;

/* Status codes of a ray. */
enum { OR_ESCAPED = 0, OR_CAPTURED = 1, OR_STEP_CAP = 2, OR_NONFINITE = 3, OR_AXIS = 4 };

/* ---- building blocks exposed for the pin tests ---- */
uint64_t or_splitmix64(uint64_t x);
int or_pixel_position(const or_camera* cam, int32_t i, int32_t j, double* alpha, double* beta);
void or_metric(double a, double m, double r, double th, double g[16]);
void or_metric_inverse(double a, double m, double r, double th, double gi[16]);
void or_metric_derivs(double a, double m, double r, double th, double dg[64]); /* [k][mu][nu] */
void or_christoffel(double a, double m, double r, double th, double G[64]);    /* [mu][al][be] */
double or_horizon(double a, double m);
double or_isco(double a);
/* Camera launch: X[4], K[4] and the camera tetrad legs e0, e_r, e_th, e_ph
 * (contravariant, tetrad[4][4] row = leg). */
int or_camera_launch(const or_camera* cam, double alpha, double beta,
                     double X[4], double K[4], double tetrad[16]);
/* Backward geodesic from (alpha, beta).  path receives up to cap+1 points of
 * 8 doubles (r, th, ph, Kt, Kr, Kth, Kph, dlam).  Returns 0, or -2 when the
 * ray needs more than cap points (path then holds the first cap+1). */
int or_trace_ray(const or_camera* cam, double alpha, double beta, int32_t cap,
                 double* path, int32_t* n_end, int32_t* status);
/* Plasma at a point: out = ne, Thetae, B, u^0..3, b^0..3 (11 doubles);
 * L_cm = G M / c^2 is the length unit (used by the snapshot's code units).
 * Returns 1 when the fluid four-velocity is valid, 0 otherwise, and 2 when
 * a snapshot's gathered primitives are not finite at a point within the
 * emission radius (the transfer then poisons the ray: status NONFINITE). */
int or_plasma(const or_model* model, const or_snapshot* snap, double a, double m,
              double r, double th, double ph, double L_cm, double out[11]);
/* Fluid-frame thermal coefficients (cgs): out = j_I j_Q j_V a_I a_Q a_V r_Q r_V. */
void or_thermal_coefficients(double ne, double thetae, double B, double nu,
                             double cos_thb, double out[8]);
/* Bessel-function ratios K0/K2 and K1/K2 at x. */
void or_bessel_ratios(double x, double* k0k2, double* k1k2);
/* Constant-coefficient polarized transfer over length w, from the matrix
 * exponential of the augmented propagation matrix.  coef = J_I J_Q J_V A_I
 * A_Q A_V R_Q R_V (U terms zero); S in/out (I, Q, U, V). */
void or_mueller_step(const double coef[8], const double S_in[4], double w, double S_out[4]);
/* General n x n matrix exponential (row-major), n <= 8. */
int or_expm(int n, const double* A, double* E);
/* Transfer along a stored path of n_end+1 points; out = camera Stokes
 * (I,Q,U,V) in cgs for the pixel direction (alpha, beta). */
int or_transfer_path(const or_camera* cam, const or_units* units, const or_model* model,
                     const or_snapshot* snap, double alpha, double beta,
                     const double* path, int32_t n_end, double S_out[4]);
/* Whole image (or the pixels listed in pix; pix == NULL: all, row-major).
 * stokes: [4][npix]; status: [npix]; nsteps: [npix].  nthreads <= 0: all. */
int or_render(const or_camera* cam, const or_units* units, const or_model* model,
              const or_snapshot* snap, int64_t npix, const int64_t* pix,
              double* stokes, uint8_t* status, int32_t* nsteps, int32_t nthreads);
/* Total flux densities (Jy) with Neumaier summation in row-major order, and
 * the maximum of Stokes I. */
void or_reduce(const or_camera* cam, const or_units* units, const double* stokes,
               double flux_jy[4], double* imax);
int or_max_threads(void);

/* Electron distributions of the nonthermal module. */
#define OR_DIST_KAPPA 0
#define OR_DIST_THERMAL 1
/* Synchrotron functions F, G, H at n points X: out[3i..3i+2]. */
void or_synchrotron_kernels(int64_t n, const double* X, double* out);
/* K_nu(x) and int_x^inf K_nu(s) ds at n points. */
void or_bessel_k(int64_t n, double nu, const double* x, double* k, double* ki);
/* The eight dimensionless integrals I_F I_G I_H A_F A_G A_H R_Q R_V of the
 * distribution at n points in[3i..3i+2] = (kappa, w, X). */
void or_kappa_integrals(int32_t dist, int64_t n, const double* in, double* out, int32_t threads);
/* Fluid-frame coefficients (cgs) of the distribution, layout of
 * or_thermal_coefficients. */
void or_kappa_coefficients(int32_t dist, double kappa, double ne, double w, double B, double nu,
                           double cos_thb, double out[8]);

#ifdef __cplusplus
}
#endif
#endif
