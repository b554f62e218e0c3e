/*
 * krt: polarized Kerr ray tracing on AMD MI355X (gfx950) -- C ABI.
 *
 * The library implements the hot path of the method of Moscibrodzka &
 * Yfantis (2023, "Prospects for ray-tracing light intensity and polarization
 * in models of accreting compact objects using a GPU"), Sec. 2.1-2.2: one ray
 * per camera pixel; a null geodesic integrated backward in time from the
 * camera with an adaptive step controlled by a parameter eps, and saved; then
 * covariant, fully polarized synchrotron transfer (Stokes I, Q, U, V carried
 * as a complex coherency matrix in the coordinate frame) integrated forward
 * along the saved path toward the camera, with plasma quantities and
 * emission / absorption / Faraday rotation and conversion coefficients
 * evaluated at every stored point.  The product is one polarized image
 * (Table 1 caption: Stokes I, Q, U, V per image).
 *
 * Conventions.  Geometry in units G = c = M = 1, Kerr-Schild coordinates
 * (t, r, theta, phi); radiative quantities in cgs.  Pixel (i, j) of an
 * nx x ny image sits at alpha = fov_x ((i + 1/2 + d_x)/nx - 1/2),
 * beta = fov_y ((j + 1/2 + d_y)/ny - 1/2) (d = SplitMix64 jitter in
 * [-1/2, 1/2) or 0); +alpha is image right (along e_phi of the static camera),
 * +beta is image up (along -e_theta).
 *
 * Memory.  Every pointer named d_* is DEVICE memory owned by the caller
 * (allocated e.g. by PyTorch on the context's device); the library never
 * frees it.  The library owns the context and its scratch memory (path store,
 * counters, tables), allocated by krt_create / krt_trace and freed by
 * krt_destroy.  No managed memory is used.
 *
 * Streams.  Every call enqueues on the context's stream (default: the null
 * stream; see krt_set_stream) and returns without waiting, except where a
 * function says it synchronises.
 *
 * Errors.  Functions return KRT_OK or an error code; krt_last_error() gives
 * a message.  All parameter checks run on the host before any launch.
 * Numerical trouble on a single ray is not an error: it is reported per
 * pixel in the status image (KRT_RAY_*) and counted in krt_stats.
 */
#ifndef KRT_H
#define KRT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KRT_ABI_VERSION 8

typedef enum {
    KRT_OK = 0,
    KRT_E_INVAL = 1,       /* invalid argument (checked on the host)          */
    KRT_E_NOMEM = 2,       /* device or host allocation failed                */
    KRT_E_HIP = 3,         /* HIP runtime error                               */
    KRT_E_STATE = 4,       /* call out of order (e.g. no model set)           */
    KRT_E_UNSUPPORTED = 5  /* valid but not supported by this library         */
} krt_status;

/* Per-pixel ray status (uint8 status image). */
enum {
    KRT_RAY_ESCAPED = 0,   /* left through r > r_cam moving outward           */
    KRT_RAY_CAPTURED = 1,  /* reached r < 1.05 r_+ (flat test mode: r < 1e-6) */
    KRT_RAY_STEP_CAP = 2,  /* hit max_steps                                   */
    KRT_RAY_NONFINITE = 3, /* non-finite state or Stokes vector               */
    KRT_RAY_AXIS = 4       /* sin(theta) < 1e-12                              */
};

typedef struct krt_ctx krt_ctx;

/* Camera and integration parameters.  Sec. 2.1 lists spin, viewing angle,
 * observing frequency, field of view and resolution; Sec. 2.2 the step
 * parameter eps.  Every struct starts with its size (set it to sizeof). */
typedef struct {
    uint32_t struct_size;
    double a;            /* spin, |a| < 1                                     */
    double incl_deg;     /* camera polar angle theta_o, 0 < theta_o < 180     */
    double phi_deg;      /* camera azimuth                                    */
    double r_cam;        /* camera radius (units of M), > 2 r_+               */
    double fov_x, fov_y; /* field of view (units of M), > 0                   */
    int32_t nx, ny;      /* resolution, >= 1                                  */
    double freq_hz;      /* observing frequency at the camera, > 0            */
    double eps;          /* step parameter, 0 < eps <= 0.5: each step changes
                            ln r, theta, ln sin(theta) and phi by about eps  */
    int32_t max_steps;   /* step cap per ray, >= 1                            */
    int32_t jitter;      /* 1: seeded jitter inside each pixel, 0: centres    */
    uint64_t seed;       /* jitter seed                                       */
    int32_t mass_factor; /* 1: Kerr; 0: flat space (test mode)                */
} krt_camera;

/* Physical units: black-hole mass and distance (Sec. 2.1: the image
 * normalisation depends on the mass-accretion-rate scale). */
typedef struct {
    uint32_t struct_size;
    double M_bh_g;       /* g, > 0                                            */
    double dist_cm;      /* cm, > 0                                           */
} krt_units;

/* Analytic ADAF-like flow (Sec. 2.1 semianalytic model; parameters are a
 * reading: n_e = n0 r^-3/2 exp(-z^2/(2 (h r)^2)), z = r cos(theta),
 * T_e = T0/r, |B| from beta = p_virial/p_mag with p_virial = n_e m_p c^2/(6 r),
 * Keplerian rotation outside the ISCO and zero angular momentum inside,
 * toroidal field). */
typedef struct {
    uint32_t struct_size;
    double n0_cgs;       /* >= 0 */
    double T0_K;         /* > 0  */
    double beta;         /* > 0  */
    double h_over_r;     /* > 0  */
    int32_t field_geom;  /* 0: toroidal (the only value supported)            */
} krt_adaf;

/* Gridded GRMHD-like snapshot on a modified Kerr-Schild grid (Sec. 2.1:
 * plasma read from precomputed 3D arrays and interpolated at every step).
 * x1 = ln r, theta = pi x2 + (1 - hslope)/2 sin(2 pi x2), x3 = phi;
 * cell-centred. */
typedef struct {
    uint32_t struct_size;
    int32_t n1, n2, n3;
    double x1_start, dx1, x2_start, dx2, x3_start, dx3;
    double hslope;
    double gamma_ad;     /* adiabatic index                                   */
    double M_unit_g;     /* mass unit: rho_unit = M_unit / L^3                */
    double R_high, R_low;
    double sigma_cut;    /* no emission where b.b/rho > sigma_cut             */
    double r_emit_max;   /* no emission beyond this radius                    */
    int32_t layout;      /* 0: [n1][n2][n3][8] (the eight fields of a cell
                            together); 1: [8][n1][n2][n3] (one array per
                            field); field order rho, u, U1..3, B1..3          */
} krt_snapshot_desc;

/* Counters of one krt_trace call. */
typedef struct {
    uint32_t struct_size;
    int64_t rays;            /* pixels traced                                 */
    int64_t total_steps;     /* sum over rays of geodesic steps               */
    int64_t status_count[5]; /* rays per KRT_RAY_* status                     */
    int32_t max_steps_seen;  /* longest ray                                   */
    int64_t long_rays;       /* rays longer than the fast path's store        */
    double kernel_ms[2];     /* device time of the wave-synchronous tracer and
                                of the long-ray tracer (HIP events)           */
    int64_t surrogate_points; /* kappa electrons: points whose coefficients
                                 came from the surrogate                      */
    int64_t exact_points;    /* kappa electrons: points evaluated with the
                                exact integrator (all of them in the exact
                                mode; the out-of-domain fallback otherwise)   */
} krt_stats;

/* ---- lifecycle ---- */

/* Version of this ABI (KRT_ABI_VERSION). */
int krt_abi_version(void);

/* The calls below follow the paper's problem statement (Sec. 2.1): the
 * inputs of one image are the model (semianalytic or GRMHD arrays), the
 * mass-accretion-rate scale, the electron-temperature prescription, the spin,
 * the viewing angle, the observing frequency, the field of view and the
 * resolution, and the step parameter of the geodesic integration (Sec. 2.2);
 * the output is one Stokes I, Q, U, V image (Table 1 caption). */

/* Creates a context on HIP device `device` (which becomes current for the
 * calling thread) and builds the library's constant tables there (the
 * Bessel-function ratios of the thermal rotativities, Sec. 2.1 Faraday
 * effects).
 * *out receives the context.  Errors: KRT_E_INVAL (bad device or NULL out),
 * KRT_E_NOMEM, KRT_E_HIP. */
krt_status krt_create(int device, krt_ctx** out);

/* Waits for the context's stream, frees everything the context owns and the
 * context itself.  NULL is accepted. */
krt_status krt_destroy(krt_ctx* ctx);

/* Borrows a hipStream_t for all later calls (NULL: the null stream).  The
 * caller keeps ownership and must keep the stream alive. */
krt_status krt_set_stream(krt_ctx* ctx, void* hip_stream);

/* Sets the physical units (default: none; krt_trace needs them): the mass
 * sets the length unit L = G M / c^2 of the path and, with the distance, the
 * flux scale of the image (Sec. 2.1, mass-accretion-rate scaling).  Errors:
 * KRT_E_INVAL (NULL, wrong struct_size, non-finite or non-positive). */
krt_status krt_set_units(krt_ctx* ctx, const krt_units* units);

/* Selects the analytic ADAF model with these parameters (Sec. 2.1: plasma
 * of a semianalytic model computed at every step along the geodesic).
 * Errors: KRT_E_INVAL (bad struct or values), KRT_E_UNSUPPORTED (field
 * geometry other than toroidal). */
krt_status krt_set_model_adaf(krt_ctx* ctx, const krt_adaf* adaf);

/* Element types of snapshot primitives. */
enum { KRT_DTYPE_F64 = 0, KRT_DTYPE_F32 = 1 };

/* Selects the snapshot model (Sec. 2.1: plasma of a GRMHD model read from
 * precomputed 3D arrays and interpolated at every step).  d_prims (device
 * memory, layout per desc,
 * element type KRT_DTYPE_F64 or KRT_DTYPE_F32: the FP32 copy halves the
 * gather traffic and is read by both transfer precisions) is borrowed until
 * the model is replaced or the context is destroyed; the caller must keep it
 * alive and unchanged meanwhile.  The library also builds, on the context's
 * stream, its table of the MKS inversion x2(theta) for desc's hslope (8 KiB
 * of device memory it owns).  Errors: KRT_E_INVAL, KRT_E_UNSUPPORTED (dtype
 * other than KRT_DTYPE_F64 / KRT_DTYPE_F32, layout other than 0 or 1),
 * KRT_E_NOMEM (the table or a layout-1 copy cannot be allocated). */
krt_status krt_set_model_snapshot(krt_ctx* ctx, const krt_snapshot_desc* desc,
                                  const void* d_prims, int dtype);

/* Arithmetic of the polarized transfer (Sec. 4 of the paper names single
 * precision as the next speed-up).  KRT_PRECISION_FP64 (default): everything
 * FP64.  KRT_PRECISION_FP32_TRANSFER: geodesics and their step control stay
 * FP64; the stored path is kept in FP32 (32 B per point: r, the signed
 * distance to the nearer pole, phi reduced to [0, 2 pi), K^mu, the step); the
 * operators of each transfer step (metric and connection, plasma,
 * coefficients, fluid tetrad, propagator) are FP32, while the coherency
 * matrix and the transport state stay FP64 and every increment is added in
 * FP64.  Applies to later krt_trace calls.  Errors: KRT_E_INVAL. */
enum { KRT_PRECISION_FP64 = 0, KRT_PRECISION_FP32_TRANSFER = 1 };
krt_status krt_set_precision(krt_ctx* ctx, int precision);

/* ---- the hot path ---- */

/* Traces the whole image (Sec. 2.1): per pixel, camera launch, backward null
 * geodesic with the eps-controlled adaptive step (stored), then the covariant
 * polarized transfer of the coherency matrix forward along the stored path
 * with plasma, emission, absorption and Faraday coefficients at every point
 * (Sec. 2.1, Sec. 2.2: the CPU code's stored-path scheme).  d_stokes: [4][ny][nx] FP64, Stokes I, Q, U, V
 * in erg s^-1 cm^-2 sr^-1 Hz^-1 at the camera.  d_status: [ny][nx] uint8
 * KRT_RAY_* (may be NULL).  Asynchronous; when out_stats is non-NULL the call
 * synchronises the stream and fills it.  Errors: KRT_E_INVAL, KRT_E_STATE
 * (no units or model), KRT_E_NOMEM, KRT_E_HIP. */
krt_status krt_trace(krt_ctx* ctx, const krt_camera* cam, double* d_stokes, uint8_t* d_status,
                     krt_stats* out_stats);

/* As krt_trace, and also writes the number of geodesic steps of every ray to
 * d_nsteps ([ny][nx] int32, may be NULL).  Same errors as krt_trace. */
krt_status krt_trace_steps(krt_ctx* ctx, const krt_camera* cam, double* d_stokes,
                           uint8_t* d_status, int32_t* d_nsteps, krt_stats* out_stats);

/* Measurement probe of the per-ray work of the image traced by krt_trace
 * (Sec. 2.2 reports the GPU's throughput; this hook lets hardware instruction
 * counters see that work without lane divergence): each listed pixel
 * (pixels: HOST array of npix row-major indices into the camera's nx x ny
 * image, copied by the call) is traced by all 64 lanes of one wavefront, with
 * the same per-ray arithmetic as krt_trace.  d_stokes: [4][npix] FP64, the
 * listed pixels' Stokes vectors (equal to krt_trace's values of those pixels).
 * out_stats (may be NULL) counts every lane: rays = 64 npix and total_steps =
 * 64 x the listed rays' steps.  Thermal electrons only.  Synchronous.
 * Errors: KRT_E_INVAL (empty list, index outside the image, bad camera),
 * KRT_E_STATE, KRT_E_UNSUPPORTED (kappa electrons), KRT_E_NOMEM (also when a
 * listed ray outgrows the path store: the probe has no long-ray pass),
 * KRT_E_HIP. */
krt_status krt_trace_probe(krt_ctx* ctx, const krt_camera* cam, const int32_t* pixels, int32_t npix,
                           double* d_stokes, krt_stats* out_stats);

/* ---- batched image libraries ---- */

/* Launch configuration of the persistent tracers (context-wide; chosen by
 * hand or by krt_autotune).  tile_w: pixels per row of the pixel tile one
 * 64-lane wave traces, 64 / tile_w rows (4, 8, 16, 32 or 64; default 8);
 * blocks_per_cu: blocks of 256 threads per compute unit in the persistent
 * grid (0: as many as fit); path_cap: points per wave slice of the path store
 * (0: KRT_PATH_CAP or 8192), longer paths continue in chunks; order: 1 (the
 * default) queues a plain image's tiles nearest the image centre first (the
 * longest rays, near the shadow's edge, start first) and a batch's groups
 * with most instances first; 0 keeps row-major tiles and the given groups;
 * 2 splits a plain image into 8 sectors of 45 degrees around its centre,
 * one per XCD, each queued centre-first and taken first by the waves of
 * that XCD (blocks dealt to the XCDs in turn), which keep a sector's
 * snapshot cells in one L2 (batches: as 1).  The order never changes an
 * image; order is validated to 0, 1 or 2 (KRT_E_INVAL otherwise). */
typedef struct {
    uint32_t struct_size;
    int32_t tile_w;
    int32_t blocks_per_cu;
    int32_t path_cap;
    int32_t order;
} krt_launch_config;

krt_status krt_set_launch_config(krt_ctx* ctx, const krt_launch_config* cfg);
krt_status krt_get_launch_config(const krt_ctx* ctx, krt_launch_config* out);

/* One image of a batch (the paper's motivation: libraries of many images of
 * one model, Sec. 1 and Sec. 4).  group: index of the camera (geometry,
 * resolution, step control) whose geodesics the image shares; freq_hz: its
 * observing frequency; M_unit_g, R_high: snapshot mass unit and electron
 * temperature ratio (0: the model's values; must be 0 for the ADAF model);
 * d_stokes: [4][ny][nx] FP64 output of the group's resolution (device memory,
 * caller-owned); d_status: [ny][nx] uint8 or NULL. */
typedef struct {
    uint32_t struct_size;
    int32_t group;
    double freq_hz;
    double M_unit_g;
    double R_high;
    double* d_stokes;
    uint8_t* d_status;
} krt_instance;

/* Traces a batch of images in one persistent launch: each queue item is one
 * tile of one group; its geodesics are integrated once (they do not depend on
 * frequency or on the plasma normalisation) and the stored path is walked once
 * per instance of the group.  Each image equals the one krt_trace would make
 * for the group camera at the instance's frequency and plasma parameters.
 * The groups' freq_hz fields are not used; all groups share the spin and mass
 * factor.  out_stats (optional) counts instance rays.  Errors: KRT_E_INVAL,
 * KRT_E_STATE, KRT_E_NOMEM, KRT_E_HIP. */
krt_status krt_trace_batch(krt_ctx* ctx, const krt_camera* groups, int32_t ngroups,
                           const krt_instance* inst, int32_t ninst, krt_stats* out_stats);

/* Launch-configuration tuner: times krt_trace_batch on a reduced form of the
 * batch (one instance per group) for a set of candidate configurations
 * (tile_w 8, 16, 32; blocks_per_cu 1, 2; path_cap 4096, 8192), sets the
 * fastest on the context and returns it.  Results are cached in the text file
 * cache_path (NULL: no cache) under a key made of the device name, its
 * compute-unit count, the precision, the model and the batch's shape, so a
 * later call with the same key only reads the file.  Synchronous. */
krt_status krt_autotune(krt_ctx* ctx, const krt_camera* groups, int32_t ngroups,
                        const krt_instance* inst, int32_t ninst, const char* cache_path,
                        krt_launch_config* out_cfg);

/* Image reduction of one Stokes I, Q, U, V image (Table 1 caption; Fig. 1
 * compares images of one model across resolutions): total flux densities
 * F_S = 1e23 dOmega sum_ij S_ij in Jy,
 * dOmega = (fov_x L / (nx D)) (fov_y L / (ny D)), L = G M / c^2, with
 * compensated summation, and the maximum of Stokes I.  d_stokes as written by
 * krt_trace for the same camera.  Synchronises the stream.  Errors:
 * KRT_E_INVAL, KRT_E_STATE (no units), KRT_E_HIP. */
krt_status krt_reduce(krt_ctx* ctx, const double* d_stokes, const krt_camera* cam,
                      double out_flux_jy[4], double* out_imax);

/* For callers that cannot allocate device memory (code under stream or graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): krt_reduce
 * with its block partials in a fixed device scratch area of the library
 * (73.9 KB per device: 1024 blocks x 9 doubles and the five results, one copy
 * per device, held until the process ends; its address is looked up once per
 * device by krt_create).  The call allocates nothing: no hipMalloc, hipFree or
 * allocating library routine; results are read back through the context's
 * pinned buffer, made by krt_create.  Any image size: the scratch's size does
 * not depend on it.  Same results as krt_reduce, bit for bit.  All calls on one
 * device share the scratch, which keeps the last call's contents (every value
 * read is written first): calls that overlap on one device (other threads, or
 * other contexts' streams) race.  Synchronises the stream.  Errors: as
 * krt_reduce; KRT_E_UNSUPPORTED for a device index of 64 or more;
 * KRT_E_STATE if the scratch address was not resolved. */
krt_status krt_reduce_noalloc(krt_ctx* ctx, const double* d_stokes, const krt_camera* cam,
                              double out_flux_jy[4], double* out_imax);

/* Message of the last error on this context (never NULL; owned by the
 * context, valid until its next call). */
const char* krt_last_error(const krt_ctx* ctx);

/* Measurement probe of the device's FP64 FMA issue rate, the ceiling the
 * tracer's roofline is set against (Sec. 2.2 compares the codes' speed; the
 * published 78.6 TFLOP/s assumes 2.4 GHz and full issue): blocks blocks of
 * 256 threads, each thread running iters rounds of 16 dependent FMA steps on
 * each of `chains` independent FP64 accumulators (chains 1, 2, 4 or 8), so
 * the launch performs blocks x 256 x iters x 16 x chains FMAs.  A grid of
 * 256 k blocks puts k waves on each SIMD.  Writes the kernel time in ms
 * (events on the context's stream) to out_ms.  Allocates and frees a
 * blocks-double buffer.  Synchronous.  Errors: KRT_E_INVAL (blocks outside
 * 1..2^20, iters outside 1..2^24, other chain counts, out_ms NULL),
 * KRT_E_NOMEM, KRT_E_HIP. */
krt_status krt_probe_fma(krt_ctx* ctx, int32_t blocks, int32_t iters, int32_t chains, double* out_ms);

/* ---- host-only checks (no device needed) ---- */

/* Validates a camera (Sec. 2.1 camera parameters, Sec. 2.2 step parameter)
 * without a context: KRT_OK or KRT_E_INVAL with a message copied into msg
 * (msg_len bytes, may be 0). */
krt_status krt_check_camera(const krt_camera* cam, char* msg, size_t msg_len);

/* ---- component hooks (same ABI; used by the parity tests) ---- */

/* Geodesic phase only (Sec. 2.1: a null geodesic per pixel from the camera,
 * adaptive step set by eps), for every pixel: d_end_state [ny][nx][8]
 * receives the last stored point (r, theta, phi, K^t, K^r, K^theta, K^phi,
 * dlam), d_nsteps [ny][nx] the step count, d_status [ny][nx] the status, and
 * d_invariant_drift [ny][nx][4] (may be NULL) the change between the camera
 * and the last point of the constants of the motion E = -K_t, L = K_phi and
 * Carter's Q = K_theta^2 + cos^2(theta) (L^2/sin^2(theta) - a^2 E^2), and the
 * null condition g(K, K) / (K^t)^2 at the last point (zero at the camera up
 * to round-off), all exact constants of the continuous geodesic, so their
 * values measure the integrator's truncation.  d_end_state is required, the
 * other outputs may be NULL.  Asynchronous.  Errors: KRT_E_INVAL. */
krt_status krt_geodesic_only(krt_ctx* ctx, const krt_camera* cam, double* d_end_state,
                             int32_t* d_nsteps, uint8_t* d_status, double* d_invariant_drift);

/* Plasma of the current model at n points (Sec. 2.1: plasma quantities at
 * every step): d_X [n][3] = (r, theta, phi) with spin a and mass factor m;
 * d_out [n][12] = (n_e, Theta_e, B, u^0..3, b^0..3, valid).  a and m are
 * arguments (not a camera) because the hook evaluates a model without a ray.
 * Needs units for the snapshot model.  Errors: KRT_E_INVAL, KRT_E_STATE. */
krt_status krt_plasma_eval(krt_ctx* ctx, int64_t n, double a, int32_t mass_factor,
                           const double* d_X, double* d_out);

/* Fluid-frame thermal coefficients at n points (Sec. 2.1: synchrotron
 * emission, self-absorption, Faraday rotation and conversion): d_in [n][5] = (n_e, Theta_e,
 * B, nu, cos theta_B); d_out [n][8] = (j_I, j_Q, j_V, alpha_I, alpha_Q,
 * alpha_V, rho_Q, rho_V), cgs. */
krt_status krt_coeffs(krt_ctx* ctx, int64_t n, const double* d_in, double* d_out);

/* Bessel-function ratios at n arguments: d_out [n][2] = (K0/K2, K1/K2)
 * (the thermal Faraday rotativities of Sec. 2.1). */
krt_status krt_bessel_ratios(krt_ctx* ctx, int64_t n, const double* d_x, double* d_out);

/* Constant-coefficient polarized update over w at n points (one step of the
 * polarized transfer of Sec. 2.1), for thermal (Kirchhoff) coefficients,
 * which is the form the thermal image uses (the general emissivity is
 * krt_mueller_general): d_coef [n][6] = (S_eq, A_I, A_Q, A_V, R_Q, R_V),
 * so that the emission is J = S_eq (A_I, A_Q, 0, A_V); d_S [n][4] in,
 * d_out [n][4] out. */
krt_status krt_mueller_step(krt_ctx* ctx, int64_t n, const double* d_coef, const double* d_S,
                            double w, double* d_out);


/* ---- Nonthermal (kappa) electrons ----------------------------------------
 * Sec. 2.1 lists the electron distribution among the model inputs and Sec. 4
 * names nonthermal electrons as the next step.  The coefficients of an
 * isotropic kappa distribution N(g) ~ g sqrt(g^2-1) (1 + (g-1)/(kappa w))^-(kappa+1)
 * (width w in place of Theta_e) follow from ultrarelativistic synchrotron
 * theory as eight dimensionless integrals over the Lorentz factor g, which
 * depend on (kappa, w, X = nu / nu_c) only, nu_c = 1.5 nu_B sin(theta_B) w^2:
 *   I_F = <F(Xg)>, I_G = <G(Xg)>, I_H = <H(Xg)/g>            (emission I, Q, V)
 *   A_F, A_G, A_H: the same with the Einstein-relation weight   (absorption)
 *   R_Q = <(2g - 1/g) Xg/(1+Xg)>, R_V = <acosh g / (g sqrt(g^2-1))>  (rotation)
 * with Xg = X w^2 / g^2 and the synchrotron functions F = X int_X K_5/3,
 * G = X K_2/3, H = X K_1/3 + int_X K_1/3.  The fluid-frame coefficients are
 * j_I = n_e c0 I_F, j_Q = n_e c0 I_G, j_V = n_e c0 (4/3) cot(theta_B) I_H,
 * alpha_S = (same with A_S) / (2 nu^2 m_e), c0 = sqrt3 e^3 B sin(theta_B) /
 * (4 pi m_e c^2), rho_Q and rho_V with the thermal prefactors times R_Q, R_V.
 */

/* Electron distribution of the traced images (krt_trace, krt_trace_steps):
 * THERMAL (default; the thermal coefficients), KAPPA_EXACT (kappa electrons
 * of index `kappa` > 2 with w = Theta_e of the model, coefficients from the
 * exact integrator at every point) or KAPPA_SURROGATE (the same, coefficients
 * from the MLP below on bf16 MFMA inside the transfer kernel, the exact
 * integrator for points outside its domain and for rays finished by the
 * long-ray kernel).  Kappa modes use FP64 transfer and the general Stokes
 * update (krt_mueller_general); KAPPA_SURROGATE needs surrogate parameters
 * (krt_mlp_set_params or krt_mlp_train).  Batched libraries stay thermal. */
#define KRT_ELECTRONS_THERMAL 0
#define KRT_ELECTRONS_KAPPA_EXACT 1
#define KRT_ELECTRONS_KAPPA_SURROGATE 2
krt_status krt_set_electrons(krt_ctx* ctx, int kind, double kappa);

/* Exact integrator: d_in [n][3] = (kappa, w, X) with kappa > 0, w > 0, X > 0
 * (device, doubles); d_out [n][8] the integrals above (device).  Trapezoid rule
 * in ln(g - 1), synchrotron functions from a Chebyshev table built on first use
 * (relative accuracy ~1e-10). */
krt_status krt_kappa_integrals(krt_ctx* ctx, int64_t n, const double* d_in, double* d_out);

/* Constant-coefficient Stokes update for a general emissivity (test hook):
 * d_coef [n][8] = (J_I, J_Q, J_V, A_I, A_Q, A_V, R_Q, R_V) with
 * A_I >= sqrt(A_Q^2 + A_V^2), d_S [n][4] in, d_out [n][4] = exp(-K w) S +
 * (int_0^w exp(-K s) ds) J over path length w >= 0. */
krt_status krt_mueller_general(krt_ctx* ctx, int64_t n, const double* d_coef, const double* d_S, double w,
                               double* d_out);

/* Learned surrogate of the eight integrals: an MLP 4 -> 64 -> 64 -> 64 -> 8
 * (SiLU) on the features x = ((kappa - 5.5)/2.5, (log10 w - 0.75)/1.25,
 * (log10 X - 2.5)/4.5, cos theta_B), whose outputs z give
 * log10 I_k = sum_j c_kj m_j(x) + mu_k + sd_k z_k: a cubic baseline in
 * (x0, x1, x2) (m_j: the 20 monomials of degree <= 3 in the order 1, x0, x1,
 * x2, x0x0, x0x1, x0x2, x1x1, x1x2, x2x2, x0x0x0, x0x0x1, x0x0x2, x0x1x1,
 * x0x1x2, x0x2x2, x1x1x1, x1x1x2, x1x2x2, x2x2x2), fitted by least squares
 * on the training set, plus the network's standardised residual.  Weight
 * matrices are used rounded to bfloat16, biases in FP32.  Parameters
 * (KRT_MLP_PARAMS floats): W1[64][4], b1[64], W2[64][64], b2[64], W3[64][64],
 * b3[64], W4[8][64], b4[8]; normalisation (KRT_MLP_NORM doubles): mu[8],
 * sd[8], c[8][20].  Domain of use: kappa in [3, 8], w in [10^-0.5, 100],
 * X in [1e-2, 1e7]. */
#define KRT_MLP_PARAMS 9160
#define KRT_MLP_NORM 176

/* Host arrays in, copied to the context (the packed inference form is rebuilt). */
krt_status krt_mlp_set_params(krt_ctx* ctx, const float* params, const double* norm);
/* Copies the current parameters and normalisation to host arrays (synchronises). */
krt_status krt_mlp_get_params(krt_ctx* ctx, float* params, double* norm);
/* Random initial weights (uniform, scaled by 1/sqrt(fan-in)), zero biases,
 * from a SplitMix64 stream of `seed`; normalisation mu = 0, sd = 1, c = 0
 * until training sets it. */
krt_status krt_mlp_init(krt_ctx* ctx, uint64_t seed);

/* Gradient of the loss L = sum over the n samples and 8 outputs of
 * (z - t)^2 / (8 n), t = (log10 integral - baseline - mu) / sd, with respect to the
 * parameters (straight through the bfloat16 rounding), for inputs d_in [n][4]
 * = (kappa, w, X, cos theta_B) and exact integrals d_integ [n][8] (device);
 * d_grad [KRT_MLP_PARAMS] (device); *out_loss = L (synchronises). */
krt_status krt_mlp_grad(krt_ctx* ctx, int64_t n, const double* d_in, const double* d_integ, float* d_grad,
                        double* out_loss);

typedef struct krt_train_config {
    uint32_t struct_size;
    int32_t epochs;        /* passes over the set                              */
    int32_t batch;         /* samples per Adam step (multiple of 32)           */
    int32_t set_norm;      /* 1: fit the baseline, mu and sd on this set;
                              0: keep the current ones                         */
    double lr_max;         /* peak Adam step                                   */
    double lr_min;         /* final step (cosine decay after a linear warm-up) */
    double warmup_frac;    /* fraction of the steps spent warming up           */
    uint64_t seed;         /* per-epoch sample order                           */
} krt_train_config;

/* Trains the MLP on the GPU with Adam (beta 0.9, 0.999, eps 1e-8) on the set
 * d_in [n][4], d_integ [n][8] (device).  n a power of two: samples are visited
 * in a fresh affine order modulo n every epoch; otherwise in the stored order.
 * *out_loss = the loss over the whole set after training (synchronises). */
krt_status krt_mlp_train(krt_ctx* ctx, int64_t n, const double* d_in, const double* d_integ,
                         const krt_train_config* cfg, double* out_loss);

/* Surrogate inference on bf16 MFMA: d_in [n][4] = (kappa, w, X, cos theta_B),
 * d_out [n][8] integrals (device).  Inputs outside the domain are evaluated
 * as they are (no fallback here). */
krt_status krt_mlp_eval(krt_ctx* ctx, int64_t n, const double* d_in, double* d_out);

#ifdef __cplusplus
}
#endif
#endif
