// HIP kernels of the polarized Kerr ray tracer (gfx950).
//
// Hot path (Sec. 2.1 of Moscibrodzka & Yfantis 2023): per pixel a backward
// geodesic, saved, then forward polarized transfer along it.  The main kernel
// is persistent and wave-synchronous: every 64-lane wavefront takes 8x8 pixel
// tiles from a device queue, integrates the 64 geodesics in lockstep
// (one RK4 step per lane per iteration) into its own slice of the path store
// (layout [point][lane][8 doubles], so each step is one coalesced 4 KiB
// write), then walks the stored points back toward the camera with all lanes
// aligned on the same point index (coalesced reads).  Rays longer than the
// slice are finished by a per-lane kernel with a full-length store.
#pragma once

#include <type_traits>

#include "krt_device.hpp"
#include "krt_f32.hpp"
#include "krt_kappa.hpp"
#include "krt_mlp.hpp"

namespace krt {

enum : uint8_t { kEscaped = 0, kCaptured = 1, kStepCap = 2, kNonFinite = 3, kAxis = 4,
                 kRunning = 254, kOverflow = 255 };

enum : int { kModelAdaf = 0, kModelSnapshot = 1 };

// Kernel modes: FP64 transfer, geodesics only, FP32 transfer operators, and
// FP64 transfer with kappa electrons (coefficients from the exact integrator
// at every point, or from the MFMA surrogate with the exact integrator
// outside its domain).
enum : int { kModeF64 = 0, kModeGeo = 1, kModeF32 = 2, kModeKapExact = 3, kModeKapMlp = 4 };

template <int kMode>
constexpr bool kKappa = kMode == kModeKapExact || kMode == kModeKapMlp;

struct TraceArgs {
    CameraDesc cam;
    double eps, r_stop, L_cm;
    double fac0;        // L_cm / freq: path length unit over the camera frequency
    int max_steps;
    int model;
    AdafDesc adaf;
    SnapDesc snap;
    const double* btab;
    const float* btab_f;   // FP32 copy of the table (set inside the kernel)
    F32Consts f32;
    // path store of the wave-synchronous kernel
    double* pool;
    int cap;            // stored points per lane slice
    int tiles_x, nbatch;
    int tile_w;         // pixels per tile row; a tile is tile_w x (64 / tile_w)
    unsigned* queue;    // [0]: next tile (or batch item)
    const int* tile_order;  // plain mode: queue position -> tile (null: row-major)
    // sectors (plain mode, nsec > 1): tile_order holds nsec + 1 sector bounds,
    // then the tiles sector by sector; squeue[s] is sector s's next position
    unsigned* squeue;
    int nsec;
    // paged extension of the wave store: chunks of `cap` points x 64 lanes,
    // taken by a wave whose rays outgrow its slice, returned after the tile
    double* chunk_pool;
    unsigned* chunk_flags;  // [nchunks], 0 = free
    int nchunks;
    // long rays
    double* long_pool;
    int long_slots;
    int32_t* overflow_list;
    int32_t* overflow_inst;  // batch mode: instance of each overflow entry
    int inst_id;
    unsigned* overflow_count;
    // batch mode: geodesic groups and image instances (null in plain mode)
    const struct GroupDev* groups;
    const struct InstDev* inst;
    int ngroups;
    // outputs
    double* stokes;     // [4][ny][nx]
    uint8_t* status;    // [ny][nx] or null
    int32_t* nsteps;    // [ny][nx] or null
    double* end_state;  // geodesic-only mode: [ny][nx][8]
    double* drift;      // geodesic-only mode: [ny][nx][4] invariant drift, or null
    unsigned long long* counters;  // steps, status[5], max steps, long rays, surrogate / exact points
    // kappa electrons
    double kappa;
    const double* syntab;       // synchrotron-function table
    const MlpPacked* mlp;       // packed surrogate
    double* phi_lds;            // per-lane phi1 tables in LDS (set inside the kernel)
    // measurement probe (plain mode): queue item t is listed pixel probe_pix[t],
    // traced by all 64 lanes of the wave; Stokes written as [4][probe_np]
    const int32_t* probe_pix;
    int probe_np;
};

// ---------------------------------------------------------------------------
// Geodesic: state y = (r, theta, phi, K^t, K^r, K^theta, K^phi).
// ---------------------------------------------------------------------------
// Derivative of the state at a point whose sin and cos of theta are given.
KRT_HD void geo_rhs_sc(double a, double m, const double y[7], double sn, double cs, double d[7]) {
    d[0] = y[4];
    d[1] = y[5];
    d[2] = y[6];
    const double K[4] = {y[3], y[4], y[5], y[6]};
    double acc[4];
    geodesic_acc_sc(a, m, y[0], sn, cs, K, acc);
    d[3] = acc[0];
    d[4] = acc[1];
    d[5] = acc[2];
    d[6] = acc[3];
}

KRT_HD void geo_rhs(double a, double m, const double y[7], double d[7]) {
    double sn, cs;
    sincos(y[1], &sn, &cs);
    geo_rhs_sc(a, m, y, sn, cs, d);
}

// sin and cos of theta + d from sin and cos of theta: the angle-addition
// formulas with Taylor series of sin d and cos d (through d^9 and d^10: below
// 1e-18 for |d| < 0.1, the step rule keeps the stage offsets near 1e-2), or a
// fresh sincos for a larger offset.
KRT_HD void sincos_shift(double th, double sn, double cs, double d, double& s2, double& c2) {
    if (fabs(d) < 0.1) {
        const double d2 = d * d;
        const double sd = d * (1.0 - d2 * (1.0 / 6.0) * (1.0 - d2 * (1.0 / 20.0) * (1.0 - d2 * (1.0 / 42.0) *
                                                                                  (1.0 - d2 * (1.0 / 72.0)))));
        const double cd = 1.0 - d2 * 0.5 * (1.0 - d2 * (1.0 / 12.0) * (1.0 - d2 * (1.0 / 30.0) *
                                                                        (1.0 - d2 * (1.0 / 56.0) *
                                                                                   (1.0 - d2 * (1.0 / 90.0)))));
        s2 = sn * cd + cs * sd;
        c2 = cs * cd - sn * sd;
    } else {
        sincos(th + d, &s2, &c2);
    }
}

// One classical RK4 step with
//   |dlam| = eps / (|K^r|/r + |K^theta| max(1, |cot theta|) + |K^phi|),
// dlam < 0: relative change of r, change of theta and phi, and relative change
// of sin(theta) bounded by eps, so steps shrink near the polar axis where the
// coordinate frame turns quickly.  (sn, cs) hold sin and cos of theta at the
// start point on entry and at the end point on return, so each point's sincos
// serves the stop test after the step and the first stage of the next one;
// the inner stages take theirs by angle addition from the start point's.
// The stage sum k1 + 2 k2 + 2 k3 + k4 is accumulated as the stages are made.
// Returns dlam.
KRT_HD double rk4_step(double a, double m, double eps, double y[7], double& sn, double& cs) {
    double k[7], ks[7], yt[7], s2, c2;
    geo_rhs_sc(a, m, y, sn, cs, k);
    const double h =
        -eps * rcp_fast(fabs(y[4]) * rcp_fast(y[0]) + fabs(y[5]) * fmax(1.0, fabs(cs * rcp_fast(sn))) + fabs(y[6]));
#pragma unroll
    for (int i = 0; i < 7; ++i) {
        ks[i] = k[i];
        yt[i] = y[i] + 0.5 * h * k[i];
    }
    sincos_shift(y[1], sn, cs, 0.5 * h * k[1], s2, c2);
    geo_rhs_sc(a, m, yt, s2, c2, k);
#pragma unroll
    for (int i = 0; i < 7; ++i) {
        ks[i] += 2.0 * k[i];
        yt[i] = y[i] + 0.5 * h * k[i];
    }
    sincos_shift(y[1], sn, cs, 0.5 * h * k[1], s2, c2);
    geo_rhs_sc(a, m, yt, s2, c2, k);
#pragma unroll
    for (int i = 0; i < 7; ++i) {
        ks[i] += 2.0 * k[i];
        yt[i] = y[i] + h * k[i];
    }
    sincos_shift(y[1], sn, cs, h * k[1], s2, c2);
    geo_rhs_sc(a, m, yt, s2, c2, k);
#pragma unroll
    for (int i = 0; i < 7; ++i) y[i] += h / 6.0 * (ks[i] + k[i]);
    sincos_polar(y[1], sn, cs);
    return h;
}

// Stop rule after step n, in order: non-finite, axis, capture, escape, cap.
// sn = sin(theta) at the new point.
KRT_HD uint8_t stop_test(const TraceArgs& A, const double y[7], double h, int n, double sn) {
    bool finite = is_finite(h);
#pragma unroll
    for (int i = 0; i < 7; ++i) finite = finite && is_finite(y[i]);
    if (!finite) return kNonFinite;
    if (sn < 1e-12) return kAxis;
    if (y[0] < A.r_stop) return kCaptured;
    if (y[0] > A.cam.r_cam && y[4] * h > 0.0) return kEscaped;
    if (n >= A.max_steps) return kStepCap;
    return kRunning;
}

// Constants of a Kerr null geodesic (Carter 1968), from the state
// y = (r, theta, phi, K^t, K^r, K^theta, K^phi): E = -K_t, L = K_phi,
// Q = K_theta^2 + cos^2(theta) (L^2 / sin^2(theta) - a^2 E^2), and the null
// condition g(K, K) / (K^t)^2.  The covariant t, theta and phi components
// are the same in Kerr-Schild and Boyer-Lindquist coordinates.
KRT_HD void geodesic_invariants(double a, double m, const double y[7], double c[4]) {
    Metric g;
    metric_eval(a, m, y[0], y[1], g);
    const double K[4] = {y[3], y[4], y[5], y[6]};
    double Kl[4];
    lower(g, K, Kl);
    const double E = -Kl[0], L = Kl[3];
    c[0] = E;
    c[1] = L;
    c[2] = Kl[2] * Kl[2] + g.c * g.c * (L * L / (g.s * g.s) - a * a * E * E);
    c[3] = (K[0] * Kl[0] + K[1] * Kl[1] + K[2] * Kl[2] + K[3] * Kl[3]) / (K[0] * K[0]);
}

// A stored point: r, theta, phi, K^t, K^r, K^theta, K^phi and the step dlam
// that reached it (64 B).
constexpr int kPointDoubles = 8;

KRT_HD void store_point(double* p, const double y[7], double h) {
    double2* q = reinterpret_cast<double2*>(p);
    q[0] = make_double2(y[0], y[1]);
    q[1] = make_double2(y[2], y[3]);
    q[2] = make_double2(y[4], y[5]);
    q[3] = make_double2(y[6], h);
}

KRT_HD void load_point(const double* p, double v[kPointDoubles]) {
    const double2* q = reinterpret_cast<const double2*>(p);
    const double2 a = q[0], b = q[1], c = q[2], d = q[3];
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
    v[4] = c.x; v[5] = c.y; v[6] = d.x; v[7] = d.y;
}

// The FP32-operator mode keeps its points in FP32 (32 B): r, the signed
// distance to the nearer pole (theta north of the equator, theta - pi south of
// it, so that sin theta keeps its relative precision at both poles), phi
// reduced to [0, 2 pi), K^t, K^r, K^theta, K^phi and the step.  Its transfer
// operators are FP32 already, and the geodesic that writes the points stays
// FP64.  Slices and chunks of the store keep 64 B per point, half used.
struct PointF {
    float r, tp, ph, K[4], d;
};

KRT_HD void store_point_f32(double* p, const double y[7], double h) {
    const double tp = y[1] > 0.5 * kPi ? y[1] - kPi : y[1];
    const double ph = y[2] - (2.0 * kPi) * floor(y[2] * (0.5 / kPi));
    float4* q = reinterpret_cast<float4*>(p);
    q[0] = make_float4((float)y[0], (float)tp, (float)ph, (float)y[3]);
    q[1] = make_float4((float)y[4], (float)y[5], (float)y[6], (float)h);
}

KRT_HD void load_point_f32(const double* p, PointF& v) {
    const float4* q = reinterpret_cast<const float4*>(p);
    const float4 a = q[0], b = q[1];
    v.r = a.x; v.tp = a.y; v.ph = a.z; v.K[0] = a.w;
    v.K[1] = b.x; v.K[2] = b.y; v.K[3] = b.z; v.d = b.w;
}

// Distance between consecutive points of the store (doubles) in mode kMode.
template <int kMode>
constexpr int kPointStride = kMode == kModeF32 ? 4 : kPointDoubles;

// ---------------------------------------------------------------------------
// Uniform parameters (spin, mass, camera, plasma model, buffers) are read
// where they are used.  Kept for the whole persistent kernel they would fill
// the scalar register file, spill into vector-register lanes and cost one
// VALU lane read per word at every use (about 300 per ray-step); a loop-
// invariant FP64 expression of them hoisted out of the loops would hold a
// vector register pair.  Instead the hot loops re-read them with scalar loads
// (scalar cache, no VALU issue) through a pointer that an empty asm makes
// opaque at each use, so neither the loads nor what is computed from them can
// be hoisted.  The source is the kernel-argument segment (the plain tracer),
// or the argument segment overlaid with a geodesic group's and an image
// instance's descriptors (the batched library); descriptors live in device
// memory that no kernel writes while a trace runs, so they may be read through
// the constant address space.
// ---------------------------------------------------------------------------
template <class T>
using ConstPtr = const __attribute__((address_space(4))) T*;

template <class T>
__device__ __forceinline__ T fresh_copy(const T* p) {
    ConstPtr<T> q = (ConstPtr<T>)p;
#if defined(__HIP_DEVICE_COMPILE__)
    asm volatile("" : "+s"(q));
#endif
    T v;
    __builtin_memcpy(&v, (const T*)q, sizeof(T));
    return v;
}

// The tables a block stages in LDS (their addresses are fixed at compile time).
struct LdsTables {
    const double* btab;
    const float* btab_f;
    const MlpPacked* mlp;
    double* phi;
};

KRT_HD void use_lds(TraceArgs& L, const LdsTables& T) {
    if (T.btab) L.btab = T.btab;
    if (T.btab_f) L.btab_f = T.btab_f;
    if (T.mlp) L.mlp = T.mlp;
    L.phi_lds = T.phi;
}

// Parameters of the plain tracer: its arguments (args: the kernel-argument
// segment, which holds them at offset 0) with the block's LDS tables.
struct PlainSource {
    const TraceArgs* args;
    LdsTables lds;
    __device__ __forceinline__ TraceArgs operator()() const {
        TraceArgs L = fresh_copy(args);
        use_lds(L, lds);
        return L;
    }
};

// ---------------------------------------------------------------------------
// Transfer state between stored points (Heun transport split in two halves):
// after point n, H = N + D_n/2 F(A_n, N) and Ns = N + D_n F(A_n, N); at point
// n-1, N = H + D_n/2 F(A_{n-1}, Ns).
// ---------------------------------------------------------------------------
struct XferState {
    Coh H, Ns;
    double Dnext;
};

// The FP32-operator transfer keeps the coherency matrix after point n in
// FP64 and the transport rate there, F(A_n, N), in FP32 (2^160-scaled): the
// predictor N + D_n F and the corrector N + D_n/2 (F + F(A_{n-1}, Ns)) are
// formed from them at point n-1 (48 instead of 64 registers of state).
struct XferStateF {
    Coh N;
    CohF F;
    double Dnext;
};

// Plasma for the radiative update: 1 with the plasma in p; 0 where the update
// leaves N unchanged (no timelike flow, or (snapshot) beyond the emission
// radius, where n_e = 0 makes every coefficient zero); 2 where the snapshot's
// gathered primitives are not finite (the ray is poisoned).
KRT_HD int plasma_at(const TraceArgs& A, double r, double th, double ph, const Metric& g,
                     Plasma& p) {
    if (A.model == kModelSnapshot) {
        if (r > A.snap.rmax) return 0;
        return snapshot_plasma(A.snap, A.cam.a, A.cam.m, r, th, ph, g, p);
    }
    return adaf_plasma(A.adaf, A.cam.a, A.cam.m, r, g, p) ? 1 : 0;
}

// Quiet NaN that poisons a ray's coherency matrix: non-finite snapshot data at
// an emitting point make the ray's Stokes vector non-finite, and its pixel is
// written as zeros with status NONFINITE.
KRT_HD double poison_nan() { return __builtin_nan(""); }

// Processes stored point n (first: the far end of the path).  On return N
// holds the coherency matrix at the point after its radiative update.
KRT_HD void transfer_point(const TraceArgs& A, const double pt[kPointDoubles], int n,
                                               bool first, XferState& st, Coh& N) {
    const double r = pt[0], th = pt[1], ph = pt[2];
    const double K[4] = {pt[3], pt[4], pt[5], pt[6]};
    const double Dn = (n == 0) ? 0.0 : fabs(pt[7]);
    Metric g;
    MetricD dr, dh;
    double sn, cs;
    sincos_polar(th, sn, cs);
    metric_eval_d_sc(A.cam.a, A.cam.m, r, sn, cs, g, dr, dh);
    double Ac[16];
    connection(g, dr, dh, K, Ac);
    double Dnext = 0.0;
    if (first) {
#pragma unroll
        for (int k = 0; k < 10; ++k) N.R[k] = 0.0;
#pragma unroll
        for (int k = 0; k < 6; ++k) N.I[k] = 0.0;
    } else {
        Dnext = st.Dnext;
        Coh F;
        transport_rhs(Ac, st.Ns, F);
        const double hh = 0.5 * Dnext;
#pragma unroll
        for (int k = 0; k < 10; ++k) N.R[k] = st.H.R[k] + hh * F.R[k];
#pragma unroll
        for (int k = 0; k < 6; ++k) N.I[k] = st.H.I[k] + hh * F.I[k];
    }

    // radiative update over w_n = (D_n + D_{n+1}) / 2
    Plasma p;
    const int pk = plasma_at(A, r, th, ph, g, p);
    if (pk == 2) N.R[0] = poison_nan();
    if (pk == 1) {
        double Kl[4];
        lower(g, K, Kl);
        const double Ku = Kl[0] * p.u[0] + Kl[1] * p.u[1] + Kl[2] * p.u[2] + Kl[3] * p.u[3];
        const double nu = A.cam.freq * (-Ku);
        const double bb = p.bb;
        const double cth =
            bb > 0.0 ? (Kl[0] * p.b[0] + Kl[1] * p.b[1] + Kl[2] * p.b[2] + Kl[3] * p.b[3]) * rsqrt_fast(bb) *
                           rcp_fast(-Ku)
                     : 0.0;
        double c[8];
        const double seq = thermal_coefficients(A.btab, p.ne, p.thetae, p.B, nu, cth, c);
        // no absorption or rotation (no plasma): the update is the identity
        // and N stays as it is
        if (c[3] != 0.0 || c[4] != 0.0 || c[5] != 0.0 || c[6] != 0.0 || c[7] != 0.0) {
            const double fac = A.fac0 * nu;
            double e1[4], l1[4], e2[4], l2[4];
            fluid_legs(g, p.u, K, p.b, bb, Ku, e1, l1, e2, l2);
            double S[4];
            coh_project(N, l1, l2, S);
            mueller_thermal(seq, fac * c[3], fac * c[4], fac * c[5], fac * c[6], fac * c[7],
                            0.5 * (Dn + Dnext), S);
            coh_rebuild(N, S, e1, e2);
        }
    }

    // (here only for n > 0: writing it also at n = 0, as the other modes do,
    // frees registers in the radiative update but gave no speed at two waves
    // per SIMD)
    if (n > 0) {
        Coh F;
        transport_rhs(Ac, N, F);
        const double hh = 0.5 * Dn;
#pragma unroll
        for (int k = 0; k < 10; ++k) {
            st.H.R[k] = N.R[k] + hh * F.R[k];
            st.Ns.R[k] = N.R[k] + Dn * F.R[k];
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            st.H.I[k] = N.I[k] + hh * F.I[k];
            st.Ns.I[k] = N.I[k] + Dn * F.I[k];
        }
        st.Dnext = Dn;
    }
}

// Fluid-frame inputs of the kappa coefficients at a stored point; returns the
// plasma_at result (1: plasma in p, nu and cth set; 0: none, the update leaves
// N unchanged; 2: non-finite data, the update poisons the ray).
KRT_HD int kappa_point(const TraceArgs& A, const double pt[kPointDoubles], Plasma& p, double& nu, double& cth) {
    const double r = pt[0], th = pt[1], ph = pt[2];
    const double K[4] = {pt[3], pt[4], pt[5], pt[6]};
    Metric g;
    double sn, cs;
    sincos_polar(th, sn, cs);
    metric_eval_sc(A.cam.a, A.cam.m, r, sn, cs, g);
    const int pk = plasma_at(A, r, th, ph, g, p);
    if (pk != 1) return pk;
    double Kl[4];
    lower(g, K, Kl);
    const double Ku = Kl[0] * p.u[0] + Kl[1] * p.u[1] + Kl[2] * p.u[2] + Kl[3] * p.u[3];
    nu = A.cam.freq * (-Ku);
    const double bb = p.bb;
    cth = bb > 0.0 ? (Kl[0] * p.b[0] + Kl[1] * p.b[1] + Kl[2] * p.b[2] + Kl[3] * p.b[3]) / (sqrt_fast(bb) * (-Ku)) : 0.0;
    return 1;
}

// transfer_point for kappa electrons: the coefficients come from the eight
// integrals I_in when use_in, else from the exact integrator (counted in
// n_exact); the update is the general constant-coefficient one.  pre: the
// plasma at the point when already evaluated, pre_kind its plasma_at result.
template <bool kPhiLds = false>
KRT_HD void transfer_point_kappa(const TraceArgs& A, const double pt[kPointDoubles], int n, bool first, XferState& st,
                                 Coh& N, const double* I_in, bool use_in, unsigned& n_exact,
                                 const Plasma* pre = nullptr, int pre_kind = 0) {
    const double r = pt[0], th = pt[1], ph = pt[2];
    const double K[4] = {pt[3], pt[4], pt[5], pt[6]};
    const double Dn = (n == 0) ? 0.0 : fabs(pt[7]);
    Metric g;
    MetricD dr, dh;
    double sn, cs;
    sincos_polar(th, sn, cs);
    metric_eval_d_sc(A.cam.a, A.cam.m, r, sn, cs, g, dr, dh);
    double Ac[16];
    connection(g, dr, dh, K, Ac);
    double Dnext = 0.0;
    if (first) {
        for (int k = 0; k < 10; ++k) N.R[k] = 0.0;
        for (int k = 0; k < 6; ++k) N.I[k] = 0.0;
    } else {
        Dnext = st.Dnext;
        Coh F;
        transport_rhs(Ac, st.Ns, F);
        const double hh = 0.5 * Dnext;
        for (int k = 0; k < 10; ++k) N.R[k] = st.H.R[k] + hh * F.R[k];
        for (int k = 0; k < 6; ++k) N.I[k] = st.H.I[k] + hh * F.I[k];
    }
    Plasma p;
    int pk;
    if (pre) {
        pk = pre_kind;
        if (pk == 1) p = *pre;
    } else {
        pk = plasma_at(A, r, th, ph, g, p);
    }
    if (pk == 2) N.R[0] = poison_nan();
    if (pk == 1) {
        double Kl[4];
        lower(g, K, Kl);
        const double Ku = Kl[0] * p.u[0] + Kl[1] * p.u[1] + Kl[2] * p.u[2] + Kl[3] * p.u[3];
        const double nu = A.cam.freq * (-Ku);
        const double bb = p.bb;
        const double cth =
            bb > 0.0 ? (Kl[0] * p.b[0] + Kl[1] * p.b[1] + Kl[2] * p.b[2] + Kl[3] * p.b[3]) / (sqrt_fast(bb) * (-Ku)) : 0.0;
        double X, sth;
        if (kappa_frame(p.ne, p.thetae, p.B, nu, cth, X, sth)) {
            double I[8];
            if (use_in) {
                for (int k = 0; k < 8; ++k) I[k] = I_in[k];
            } else {
                kappa_integrals(A.syntab, A.kappa, p.thetae, X, I);
                ++n_exact;
            }
            double c[8];
            kappa_physical(I, p.ne, p.B, nu, cth, sth, c);
            bool zero = true;
            for (int k = 0; k < 8; ++k) zero = zero && c[k] == 0.0;
            if (!zero) {
                // invariant forms: J = (L / nu_obs) j / nu^2, A = (L / nu_obs) nu alpha
                const double fa = A.fac0 * nu;
                const double fj = A.fac0 / (nu * nu);
                double e1[4], l1[4], e2[4], l2[4];
                fluid_legs(g, p.u, K, p.b, bb, Ku, e1, l1, e2, l2);
                double S[4];
                coh_project(N, l1, l2, S);
                if constexpr (kPhiLds) {
                    // this lane's slice of its wave's LDS block [22][64]
                    LdsLaneTab t{(__attribute__((address_space(3))) double*)A.phi_lds +
                                 (threadIdx.x >> 6) * (22 * 64) + (threadIdx.x & 63)};
                    mueller_general(fj * c[0], fj * c[1], fj * c[2], fa * c[3], fa * c[4], fa * c[5], fa * c[6],
                                    fa * c[7], 0.5 * (Dn + Dnext), S, t);
                } else {
                    mueller_general(fj * c[0], fj * c[1], fj * c[2], fa * c[3], fa * c[4], fa * c[5], fa * c[6],
                                    fa * c[7], 0.5 * (Dn + Dnext), S);
                }
                coh_rebuild(N, S, e1, e2);
            }
        }
    }
    {   // also at n = 0 (D_0 = 0): the state is always written, so that the
        // incoming state is dead during the radiative update (55 fewer live
        // registers there than with the write skipped at n = 0)
        Coh F;
        transport_rhs(Ac, N, F);
        const double hh = 0.5 * Dn;
        for (int k = 0; k < 10; ++k) {
            st.H.R[k] = N.R[k] + hh * F.R[k];
            st.Ns.R[k] = N.R[k] + Dn * F.R[k];
        }
        for (int k = 0; k < 6; ++k) {
            st.H.I[k] = N.I[k] + hh * F.I[k];
            st.Ns.I[k] = N.I[k] + Dn * F.I[k];
        }
        st.Dnext = Dn;
    }
}

// Mixed-precision version of transfer_point: the operators at the point in
// FP32, the coherency matrix and the Heun state in FP64, every increment
// formed in FP32 (scaled by 2^160) and added in FP64.  The radiative update
// adds the coherency matrix of the Stokes increment on the fluid legs.
KRT_HD void transfer_point_f32(const TraceArgs& A, const PointF& pt, int n, bool first, XferStateF& st,
                               Coh& N) {
    const F32Consts& C = A.f32;
    // sin and cos of theta: from the distance t0 to the nearer pole, reduced
    // in FP64 to [0, pi/4] (about pi/2 beyond pi/4), Taylor series in FP32
    // (through t^9 and t^10: truncation below 2e-10 for t <= pi/4)
    const bool south = pt.tp < 0.0f;
    const double t0 = fabs((double)pt.tp);
    const double thd = south ? kPi - t0 : t0;
    const bool upper = t0 > 0.25 * kPi;
    const float t = (float)(upper ? 0.5 * kPi - t0 : t0), t2 = t * t;
    const float sn_t = t * (1.0f + t2 * (-1.0f / 6.0f + t2 * (1.0f / 120.0f + t2 * (-1.0f / 5040.0f + t2 * (1.0f / 362880.0f)))));
    const float cs_t = 1.0f + t2 * (-0.5f + t2 * (1.0f / 24.0f + t2 * (-1.0f / 720.0f + t2 * (1.0f / 40320.0f + t2 * (-1.0f / 3628800.0f)))));
    const float s = upper ? cs_t : sn_t;
    float c = upper ? sn_t : cs_t;
    if (south) c = -c;
    const float r = pt.r;
    const float K[4] = {pt.K[0], pt.K[1], pt.K[2], pt.K[3]};
    const double Dn = (n == 0) ? 0.0 : fabs((double)pt.d);
    MetricF g;
    MetricDF dr, dh;
    metric_d_f(C.a, C.m, r, s, c, g, dr, dh);
    float Ac[16];
    connection_f(g, dr, dh, K, Ac);
    double Dnext = 0.0;
    if (first) {
#pragma unroll
        for (int k = 0; k < 10; ++k) N.R[k] = 0.0;
#pragma unroll
        for (int k = 0; k < 6; ++k) N.I[k] = 0.0;
    } else {
        Dnext = st.Dnext;
        CohF Ns, F;
        to_scaled_f(st.N, Ns);
        const float Df = (float)Dnext;
#pragma unroll
        for (int k = 0; k < 10; ++k) Ns.R[k] += Df * st.F.R[k];
#pragma unroll
        for (int k = 0; k < 6; ++k) Ns.I[k] += Df * st.F.I[k];
        transport_rhs_f(Ac, Ns, F);
        const double hh = 0.5 * Dnext * kIScaleInv;
#pragma unroll
        for (int k = 0; k < 10; ++k) N.R[k] = st.N.R[k] + hh * ((double)st.F.R[k] + (double)F.R[k]);
#pragma unroll
        for (int k = 0; k < 6; ++k) N.I[k] = st.N.I[k] + hh * ((double)st.F.I[k] + (double)F.I[k]);
    }

    PlasmaF p;
    int pk = 0;
    if (A.model == kModelSnapshot) {
        const SnapDesc& q = A.snap;
        double X2 = ((double)pt.ph - q.x3s) * q.idx3 - 0.5;
        X2 -= q.n3 * floor(X2 * q.in3);
        // no plasma beyond the emission radius (n_e = 0: every coefficient zero)
        if ((double)r <= q.rmax)
            pk = q.prims_f ? snapshot_plasma_f(C, q.prims_f, q.n1, q.n2, q.n3, r, (float)thd, (float)X2, g, p)
                           : snapshot_plasma_f(C, q.prims, q.n1, q.n2, q.n3, r, (float)thd, (float)X2, g, p);
    } else {
        pk = adaf_plasma_f(C, r, g, p) ? 1 : 0;
    }
    if (pk == 2) N.R[0] = poison_nan();
    if (pk == 1) {
        float Kl[4];
        lower_f(g, K, Kl);
        const float Ku = Kl[0] * p.u[0] + Kl[1] * p.u[1] + Kl[2] * p.u[2] + Kl[3] * p.u[3];
        const float gz = -Ku;  // nu / nu_cam
        const float bb = dot_f(g, p.b, p.b);
        // (b.b below 1e-30 counts as no field: the hardware reciprocal square
        // root does not take subnormal inputs)
        const float cth = bb > 1e-30f ? (Kl[0] * p.b[0] + Kl[1] * p.b[1] + Kl[2] * p.b[2] + Kl[3] * p.b[3]) *
                                          rsqrtf_fast(bb) * rcpf_fast(gz)
                                    : 0.0f;
        float co[5];
        const float seq = thermal_f(C, A.btab_f, p.ne, p.thetae, p.B, gz, cth, co);
        if (co[0] != 0.0f || co[1] != 0.0f || co[2] != 0.0f || co[3] != 0.0f || co[4] != 0.0f) {
            // invariant coefficients (x L nu / nu_cam) times the step length
            const float w = (float)(0.5 * (Dn + Dnext)) * C.L * gz;
            float e1[4], l1[4], e2[4], l2[4];
            fluid_legs_f(g, p.u, K, p.b, Ku, e1, l1, e2, l2);
            CohF Nf;
            to_scaled_f(N, Nf);
            float S[4], dS[4];
            coh_project_f(Nf, l1, l2, S);
            mueller_delta_f(seq, co[0] * w, co[1] * w, co[2] * w, co[3] * w, co[4] * w, S, dS);
            coh_add_delta_f(N, dS, e1, e2);
        }
    }

    {   // also at n = 0 (D_0 = 0): the state is always written, so that the
        // incoming state is dead during the radiative update
        CohF Nf;
        to_scaled_f(N, Nf);
        transport_rhs_f(Ac, Nf, st.F);
        st.N = N;
        st.Dnext = Dn;
    }
}

// Camera output: project N on the pixel's screen legs, times nu_obs^3.
KRT_HD void camera_output(const TraceArgs& A, double alpha, double beta,
                                              const Coh& N, double S[4]) {
    Metric g;
    metric_eval(A.cam.a, A.cam.m, A.cam.r_cam, A.cam.th, g);
    double ex[4], ey[4], lx[4], ly[4];
    screen_legs(A.cam, g, alpha, beta, ex, ey);
    lower(g, ex, lx);
    lower(g, ey, ly);
    coh_project(N, lx, ly, S);
    const double nu3 = A.cam.freq * A.cam.freq * A.cam.freq;
    for (int k = 0; k < 4; ++k) S[k] *= nu3;
}

// Writes one pixel; a non-finite Stokes vector is written as zeros with
// status NONFINITE.  Returns the status written (the one the counters take).
__device__ __forceinline__ uint8_t write_pixel(const TraceArgs& A, int pix, double S[4], uint8_t st,
                                               int nst) {
    const bool ok = is_finite(S[0]) && is_finite(S[1]) && is_finite(S[2]) && is_finite(S[3]);
    if (!ok) {
        S[0] = S[1] = S[2] = S[3] = 0.0;
        st = kNonFinite;
    }
    if (A.probe_pix) {   // the 64 copies are equal: lane 0 writes
        if ((threadIdx.x & 63) == 0)
            for (int k = 0; k < 4; ++k) A.stokes[(size_t)k * A.probe_np + pix] = S[k];
        return st;
    }
    const size_t np = (size_t)A.cam.nx * A.cam.ny;
    for (int k = 0; k < 4; ++k) A.stokes[k * np + pix] = S[k];
    if (A.status) A.status[pix] = st;
    if (A.nsteps) A.nsteps[pix] = nst;
    return st;
}

// Wave-level accounting of finished rays (one atomic per counter per wave).
__device__ __forceinline__ void account(const TraceArgs& A, bool valid, uint8_t st, int nst) {
    unsigned long long steps = valid ? (unsigned long long)nst : 0ULL;
    unsigned long long mx = steps;
    for (int off = 32; off >= 1; off >>= 1) {
        steps += __shfl_xor(steps, off);
        const unsigned long long o = __shfl_xor(mx, off);
        mx = o > mx ? o : mx;
    }
    unsigned long long cnt[6];
    for (int s = 0; s < 5; ++s) cnt[s] = __popcll(__ballot(valid && st == s));
    cnt[5] = __popcll(__ballot(valid && st == kOverflow));
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&A.counters[0], steps);
        for (int s = 0; s < 5; ++s)
            if (cnt[s]) atomicAdd(&A.counters[1 + s], cnt[s]);
        atomicMax(&A.counters[6], mx);
        if (cnt[5]) atomicAdd(&A.counters[7], cnt[5]);
    }
}

// Chunks of the paged path store one wave may hold for one tile: with the
// default 8192-point slice, 6 chunks cover the 50 000-step cap.
constexpr int kMaxChunks = 6;

// Called together by the active lanes of a wave (all at the same point index)
// whose slice is full: the first active lane takes a free chunk and records
// it in the wave's LDS list at position k; returns its index (-1: none free).
__device__ __forceinline__ int take_chunk(const TraceArgs& A, int* wchunks, int k, unsigned hint) {
    const unsigned long long act = __ballot(1);
    const int leader = __ffsll((unsigned long long)act) - 1;
    int id = -1;
    if ((int)(threadIdx.x & 63) == leader) {
        for (int t = 0; t < A.nchunks; ++t) {
            const int c = (int)((hint + (unsigned)t) % (unsigned)A.nchunks);
            if (atomicCAS(&A.chunk_flags[c], 0u, 1u) == 0u) {
                id = c;
                break;
            }
        }
        if (id >= 0) wchunks[k] = id;
    }
    return __builtin_amdgcn_readfirstlane(id);
}

// Address of stored point m of this lane: the wave's slice for m < cap, then
// the wave's chunks in the order taken.
// Slices and chunks are laid out for 64 B points; points are kS doubles apart.
template <int kS>
__device__ __forceinline__ const double* point_addr(const TraceArgs& A, const double* slot,
                                                   const int* wchunks, int m, int lane) {
    if (m < A.cap) return slot + ((size_t)m * 64 + lane) * kS;
    const int k = m / A.cap - 1;
    const int c = wchunks[k];
    return A.chunk_pool + (size_t)c * A.cap * 64 * kPointDoubles + ((size_t)(m - (k + 1) * A.cap) * 64 + lane) * kS;
}

// Surrogate and exact-integrator point counts of a wave, added once per tile.
__device__ __forceinline__ void kappa_account(const TraceArgs& A, unsigned n_mlp, unsigned n_exact) {
    unsigned long long a = n_mlp, b = n_exact;
    for (int off = 32; off >= 1; off >>= 1) {
        a += __shfl_xor(a, off);
        b += __shfl_xor(b, off);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&A.counters[8], a);
        atomicAdd(&A.counters[9], b);
    }
}

// Transfer phase of one tile (all lanes on the same point index, far end
// first), output and accounting.  Rays that overflowed the store are queued
// for the long-ray kernel (with their instance in batch mode).
// src() gives the parameters (read where they are used).
template <int kMode, class Src>
__device__ __forceinline__ void trace_transfer(const Src& src, double* slot, const int* wchunks,
                                               int lane, bool valid, int pix, double alpha, double beta,
                                               uint8_t st, int n) {
    if (valid && st == kOverflow) {
        const TraceArgs A = src();
        const unsigned k = atomicAdd(A.overflow_count, 1u);
        A.overflow_list[k] = pix;
        if (A.overflow_inst) A.overflow_inst[k] = A.inst_id;
    }

    // ---- transfer: all lanes on the same point index, far end first ----
    const bool xfer = valid && st != kOverflow;
    // a path whose last point is non-finite or lies on the polar axis (where
    // the coordinate frame is singular) is transferred over the points before it
    const int n_end = xfer ? ((st == kNonFinite || st == kAxis) ? n - 1 : n) : -1;
    int nred = n_end;
    for (int off = 32; off >= 1; off >>= 1) {
        const int o = __shfl_xor(nred, off);
        nred = o > nred ? o : nred;
    }
    const int nmax = __builtin_amdgcn_readfirstlane(nred);
    typename std::conditional<kMode == kModeF32, XferStateF, XferState>::type xs;
    Coh N;
    for (int k = 0; k < 10; ++k) N.R[k] = 0.0;
    for (int k = 0; k < 6; ++k) N.I[k] = 0.0;
    unsigned n_mlp = 0, n_exact = 0;
    // The exact-kappa mode (one wave per SIMD, registers to spare) loads each
    // stored point one point ahead; in the thermal modes, with two or three
    // waves per SIMD covering the load, it gains nothing.
    constexpr bool kPrefetch = kMode == kModeKapExact;
    double nxt[kPointDoubles] = {};
    if (kPrefetch && nmax >= 0 && nmax <= n_end) load_point(point_addr<kPointDoubles>(src(), slot, wchunks, nmax, lane), nxt);
    for (int m = nmax; m >= 0; --m) {
        const TraceArgs A = src();
        if constexpr (kMode == kModeKapMlp) {
            // surrogate inputs of this lane's point (in-domain points only),
            // the network for the whole wave, then the update
            float f[4] = {0.0f, 0.0f, 0.0f, 0.0f};
            bool want = false, fall = false;
            int pk = 0;
            double Xp = 0.0;
            Plasma p;
            if (m <= n_end) {
                double pt[kPointDoubles];
                load_point(point_addr<kPointDoubles>(A, slot, wchunks, m, lane), pt);
                double nu, cth, sth;
                pk = kappa_point(A, pt, p, nu, cth);
                if (pk == 1 && kappa_frame(p.ne, p.thetae, p.B, nu, cth, Xp, sth)) {
                    if (mlp_in_domain(A.kappa, p.thetae, Xp)) {
                        mlp_features(A.kappa, p.thetae, Xp, cth, f);
                        want = true;
                    } else {
                        fall = true;
                    }
                }
            }
            double I[8];
            if (__ballot(want) != 0ull) mlp_wave(A.mlp, f, I);
            // points outside the surrogate's domain: the exact integrator, one
            // point at a time with the whole wave on its quadrature nodes
            unsigned long long fb = __ballot(fall);
            while (fb != 0ull) {
                const int srcl = __ffsll(fb) - 1;
                fb &= fb - 1ull;
                const double w_s = __shfl(p.thetae, srcl), X_s = __shfl(Xp, srcl);
                double Iw[8];
                kappa_integrals_wave(A.syntab, A.kappa, w_s, X_s, Iw);
                if (lane == srcl)
                    for (int k = 0; k < 8; ++k) I[k] = Iw[k];
            }
            if (m <= n_end) {
                double pt[kPointDoubles];
                load_point(point_addr<kPointDoubles>(A, slot, wchunks, m, lane), pt);
                n_mlp += want ? 1u : 0u;
                n_exact += fall ? 1u : 0u;
                transfer_point_kappa<true>(A, pt, m, m == n_end, xs, N, I, want || fall, n_exact, &p, pk);
            }
        } else if constexpr (kMode == kModeF32) {
            if (m > n_end) continue;
            PointF pt;
            load_point_f32(point_addr<kPointStride<kMode>>(A, slot, wchunks, m, lane), pt);
            transfer_point_f32(A, pt, m, m == n_end, xs, N);
        } else {
            double pt[kPointDoubles];
            if constexpr (kPrefetch) {
                // the next point (m - 1) is loaded while this one is processed
#pragma unroll
                for (int k = 0; k < kPointDoubles; ++k) pt[k] = nxt[k];
                if (m >= 1 && m - 1 <= n_end) load_point(point_addr<kPointDoubles>(A, slot, wchunks, m - 1, lane), nxt);
                if (m > n_end) continue;
            } else {
                if (m > n_end) continue;
                load_point(point_addr<kPointDoubles>(A, slot, wchunks, m, lane), pt);
            }
            if constexpr (kMode == kModeKapExact)
                transfer_point_kappa(A, pt, m, m == n_end, xs, N, nullptr, false, n_exact);
            else
                transfer_point(A, pt, m, m == n_end, xs, N);
        }
    }
    const TraceArgs A = src();
    if constexpr (kKappa<kMode>) kappa_account(A, n_mlp, n_exact);
    uint8_t st_out = st;
    if (xfer) {
        double S[4];
        camera_output(A, alpha, beta, N, S);
        st_out = write_pixel(A, pix, S, st, n);
    }
    // counted with the status written (a non-finite Stokes vector turns the
    // geodesic's status into NONFINITE); overflow rays are counted by the
    // long-ray kernel
    account(A, valid, st_out, n);
}

// Pixel of a lane in tile `tile` of an image with tiles_x tiles per row; a
// tile is tile_w pixels wide and 64 / tile_w rows high.
__device__ __forceinline__ void tile_pixel(int tiles_x, int tile_w, int tile, int lane, int& i, int& j) {
    const int th = 64 / tile_w;
    i = (tile % tiles_x) * tile_w + lane % tile_w;
    j = (tile / tiles_x) * th + lane / tile_w;
}

// Geodesic phase of one tile: camera launch and RK4 steps in lockstep, every
// point stored in the wave's slice, then in chunks of the paged store (kStore),
// or only the end state kept; kCompact: in the FP32-operator mode's format.
// Returns the number of chunks the wave holds.
template <bool kStore, bool kCompact, class Src>
__device__ __forceinline__ int geodesic_phase(const Src& src, bool valid, int i, int j, double* slot,
                                              int* wchunks, size_t wave, int lane, double& alpha,
                                              double& beta, double y[7], double& hlast, uint8_t& st,
                                              int& n) {
    alpha = 0.0;
    beta = 0.0;
    {
        const CameraDesc C = src().cam;
        pixel_position(C, valid ? i : 0, valid ? j : 0, alpha, beta);
        double X[4], K[4];
        camera_launch(C, alpha, beta, X, K);
        y[0] = X[1]; y[1] = X[2]; y[2] = X[3];
        y[3] = K[0]; y[4] = K[1]; y[5] = K[2]; y[6] = K[3];
    }
    double sn, cs;
    sincos_polar(y[1], sn, cs);
    constexpr int kS = kCompact ? 4 : kPointDoubles;
    if (kStore && valid) {
        if constexpr (kCompact)
            store_point_f32(slot + (size_t)lane * kS, y, 0.0);
        else
            store_point(slot + (size_t)lane * kS, y, 0.0);
    }

    st = valid ? kRunning : kEscaped;
    n = 0;
    hlast = 0.0;
    // store of points [cstart, cstart + cap): the slice, then chunks; the
    // lanes still stepping all sit at the same n, so nch, cstart and cbase
    // agree among them
    int nch = 0, cstart = 0;
    double* cbase = slot;
    while (st == kRunning) {
        const TraceArgs A = src();
        const double h = rk4_step(A.cam.a, A.cam.m, A.eps, y, sn, cs);
        ++n;
        hlast = h;
        if (kStore) {
            if (n == cstart + A.cap) {
                const int id = (nch < kMaxChunks && A.nchunks > 0)
                                   ? take_chunk(A, wchunks, nch, (unsigned)wave * 7u + (unsigned)nch)
                                   : -1;
                if (id < 0) {  // no chunk: the long-ray kernel redoes these rays
                    st = kOverflow;
                    continue;
                }
                ++nch;
                cstart += A.cap;
                cbase = A.chunk_pool + (size_t)id * A.cap * 64 * kPointDoubles;
            }
            double* p = cbase + ((size_t)(n - cstart) * 64 + lane) * kS;
            if constexpr (kCompact)
                store_point_f32(p, y, h);
            else
                store_point(p, y, h);
        }
        st = stop_test(A, y, h, n, sn);
    }
    int nch_w = nch;
    for (int off = 32; off >= 1; off >>= 1) {
        const int o = __shfl_xor(nch_w, off);
        nch_w = o > nch_w ? o : nch_w;
    }
    return __builtin_amdgcn_readfirstlane(nch_w);
}

// The Bessel-ratio table (15 KiB in FP64, 7.5 KiB in FP32) is read at every
// transfer point with lane-dependent panels: every block stages it in LDS.
template <int kMode>
__device__ __forceinline__ void stage_table(TraceArgs& A, double* s_btab, float* s_btab_f) {
    constexpr int kTab = kBesPanels * 2 * kBesCoef;
    if (kMode == kModeF64) {
        for (int k = threadIdx.x; k < kTab; k += blockDim.x) s_btab[k] = A.btab[k];
        __syncthreads();
        A.btab = s_btab;
    } else if (kMode == kModeF32) {
        for (int k = threadIdx.x; k < kTab; k += blockDim.x) s_btab_f[k] = (float)A.btab[k];
        __syncthreads();
        A.btab_f = s_btab_f;
    }
}

// ---------------------------------------------------------------------------
// Persistent wave-synchronous tracer.  kMode: FP64 transfer, FP32 transfer
// operators, or (kModeGeo) the geodesic phase only, writing the end state (no
// store, no transfer).  Two waves per SIMD (at most 256 registers per lane):
// with one, the FP64 dependency chains of a single wave leave the vector ALU
// idle.  The FP32-operator mode (fewer than 168 registers) runs three; the
// FP64 mode (256) would spill heavily at the 168 that three allow.  The kappa
// modes run one.
// ---------------------------------------------------------------------------
template <int kMode>
__global__ __launch_bounds__(256, kMode == kModeKapExact ? 1 : (kMode == kModeF32 ? 3 : 2)) void trace_waves(TraceArgs A) {
    constexpr bool kGeoOnly = kMode == kModeGeo;
    constexpr int kTab = kBesPanels * 2 * kBesCoef;
    __shared__ double s_btab[kMode == kModeF64 ? kTab : 1];
    __shared__ float s_btab_f[kMode == kModeF32 ? kTab : 1];
    __shared__ int4 s_mlp[kMode == kModeKapMlp ? sizeof(MlpPacked) / 16 : 1];
    // the surrogate kernel (two waves per SIMD) keeps the general update's
    // Taylor table in LDS rather than in registers
    __shared__ double s_phi[kMode == kModeKapMlp ? 4 * 22 * 64 : 1];
    stage_table<kMode>(A, s_btab, s_btab_f);
    if constexpr (kMode == kModeKapMlp) {
        const int4* src = reinterpret_cast<const int4*>(A.mlp);
        for (int k = threadIdx.x; k < (int)(sizeof(MlpPacked) / 16); k += blockDim.x) s_mlp[k] = src[k];
        __syncthreads();
        A.mlp = reinterpret_cast<const MlpPacked*>(s_mlp);
    }
    const PlainSource src{(const TraceArgs*)__builtin_amdgcn_kernarg_segment_ptr(),
                          {kMode == kModeF64 ? s_btab : nullptr, kMode == kModeF32 ? s_btab_f : nullptr,
                           kMode == kModeKapMlp ? reinterpret_cast<const MlpPacked*>(s_mlp) : nullptr,
                           kMode == kModeKapMlp ? s_phi : nullptr}};
    const int lane = threadIdx.x & 63;
    // the wave index is uniform: read it from the first lane so that the
    // slice address lives in scalar registers
    const size_t wave = (size_t)blockIdx.x * (blockDim.x >> 6) +
                        (size_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    __shared__ int s_chunks[4][kMaxChunks];
    int* wchunks = s_chunks[threadIdx.x >> 6];
    // With sectors, blocks are dealt to the XCDs in turn (block b on XCD
    // b mod 8), so a wave starts on the sector of its XCD, whose tiles lie
    // together on the image (and their snapshot cells in that XCD's L2), and
    // moves on to the next sectors when its own is drained.
    int sec = A.nsec > 1 ? (int)(blockIdx.x % (unsigned)A.nsec) : 0;
    int drained = 0;
    for (;;) {
        const TraceArgs A = src();
        const int nsec = A.nsec;
        double* slot = A.pool + wave * (size_t)A.cap * 64 * kPointDoubles;
        // One queue ticket per wave, taken without a lane-divergent branch:
        // every lane adds 0 except lane 0, and the wave uses lane 0's ticket
        // as a scalar, so the loop exit below is wave-uniform.
        unsigned* q = nsec > 1 ? A.squeue + sec : A.queue;
        const unsigned ticket = atomicAdd(q, lane == 0 ? 1u : 0u);
        const int pos = __builtin_amdgcn_readfirstlane((int)ticket);
        int tile;
        if (nsec > 1) {
            const int b0 = A.tile_order[sec], b1 = A.tile_order[sec + 1];
            if (pos >= b1 - b0) {
                if (++drained == nsec) break;
                sec = sec + 1 == nsec ? 0 : sec + 1;
                continue;
            }
            tile = A.tile_order[nsec + 1 + b0 + pos];
        } else {
            if (pos >= A.nbatch) break;
            tile = A.tile_order ? A.tile_order[pos] : pos;
        }
        int i, j;
        tile_pixel(A.tiles_x, A.tile_w, tile, lane, i, j);
        if (A.probe_pix) {
            const int p = A.probe_pix[tile];
            i = p % A.cam.nx;
            j = p / A.cam.nx;
        }
        const bool valid = i < A.cam.nx && j < A.cam.ny;
        const int pix = A.probe_pix ? tile : j * A.cam.nx + i;
        double alpha, beta, hlast, y[7];
        uint8_t st;
        int n;
        const int nch_w =
            geodesic_phase<!kGeoOnly, kMode == kModeF32>(src, valid, i, j, slot, wchunks, wave, lane, alpha, beta, y,
                                                         hlast, st, n);
        if (kGeoOnly) {
            const TraceArgs A = src();
            if (valid) {
                double* e = A.end_state + (size_t)pix * 8;
                for (int k = 0; k < 7; ++k) e[k] = y[k];
                e[7] = hlast;
                if (A.status) A.status[pix] = st;
                if (A.nsteps) A.nsteps[pix] = n;
                if (A.drift) {
                    // constants of the motion at the camera (the launch state,
                    // recomputed) and at the last point
                    double y0[7], c0[4], c1[4];
                    const CameraDesc C = A.cam;
                    double X[4], K[4];
                    camera_launch(C, alpha, beta, X, K);
                    y0[0] = X[1]; y0[1] = X[2]; y0[2] = X[3];
                    y0[3] = K[0]; y0[4] = K[1]; y0[5] = K[2]; y0[6] = K[3];
                    geodesic_invariants(C.a, C.m, y0, c0);
                    geodesic_invariants(C.a, C.m, y, c1);
                    double* d = A.drift + (size_t)pix * 4;
                    for (int k = 0; k < 4; ++k) d[k] = c1[k] - c0[k];
                }
            }
            account(A, valid, st, n);
        } else {
            trace_transfer<kMode>(src, slot, wchunks, lane, valid, pix, alpha, beta, st, n);
            const TraceArgs A = src();
            if (lane == 0)
                for (int k = 0; k < nch_w; ++k) atomicExch(&A.chunk_flags[wchunks[k]], 0u);
        }
    }
}

// ---------------------------------------------------------------------------
// Batched image library: geodesic groups (one camera geometry and resolution
// each) and image instances (frequency, snapshot mass unit and R_high, output
// image) of those groups.  One queue item is one tile of one group: the wave
// traces the tile's geodesics once and walks the stored path once per
// instance of the group.
// ---------------------------------------------------------------------------
struct GroupDev {
    CameraDesc cam;           // geometry (cam.freq unused)
    double eps, r_stop;
    int max_steps;
    int tiles_x;
    int item_begin, item_end; // queue items (tiles) of the group
    int inst_begin, inst_end; // its instances in the instance array
};

struct InstDev {
    double freq, fac0;
    double rho_unit, B_unit, Rhigh;  // snapshot model
    F32Consts f32;
    double* stokes;
    uint8_t* status;
    int group;
};

KRT_HD void apply_group(TraceArgs& L, const GroupDev& G) {
    L.cam = G.cam;
    L.eps = G.eps;
    L.r_stop = G.r_stop;
    L.max_steps = G.max_steps;
    L.tiles_x = G.tiles_x;
}

KRT_HD void apply_instance(TraceArgs& L, const InstDev& I, int q) {
    L.cam.freq = I.freq;
    L.fac0 = I.fac0;
    L.snap.rho_unit = I.rho_unit;
    L.snap.B_unit = I.B_unit;
    L.snap.Rhigh = I.Rhigh;
    L.f32 = I.f32;
    L.stokes = I.stokes;
    L.status = I.status;
    L.nsteps = nullptr;
    L.inst_id = q;
}

// Parameters of a batch item: the kernel arguments overlaid with geodesic
// group g and (q >= 0) image instance q, read where they are used.
struct BatchSource {
    PlainSource base;
    int g, q;
    __device__ __forceinline__ TraceArgs operator()() const {
        TraceArgs L = base();
        apply_group(L, fresh_copy(L.groups + g));
        if (q >= 0) apply_instance(L, fresh_copy(L.inst + q), q);
        return L;
    }
};

template <int kMode>
__global__ __launch_bounds__(256, 2) void trace_batch(TraceArgs A) {
    constexpr int kTab = kBesPanels * 2 * kBesCoef;
    __shared__ double s_btab[kMode == kModeF64 ? kTab : 1];
    __shared__ float s_btab_f[kMode == kModeF32 ? kTab : 1];
    stage_table<kMode>(A, s_btab, s_btab_f);
    const PlainSource base{(const TraceArgs*)__builtin_amdgcn_kernarg_segment_ptr(),
                           {kMode == kModeF64 ? s_btab : nullptr, kMode == kModeF32 ? s_btab_f : nullptr,
                            nullptr}};
    const int lane = threadIdx.x & 63;
    // the wave index is uniform: read it from the first lane so that the
    // slice address lives in scalar registers
    const size_t wave = (size_t)blockIdx.x * (blockDim.x >> 6) +
                        (size_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    __shared__ int s_chunks[4][kMaxChunks];
    int* wchunks = s_chunks[threadIdx.x >> 6];
    for (;;) {
        const TraceArgs A = base();
        double* slot = A.pool + wave * (size_t)A.cap * 64 * kPointDoubles;
        const unsigned ticket = atomicAdd(A.queue, lane == 0 ? 1u : 0u);
        const int item = __builtin_amdgcn_readfirstlane((int)ticket);
        if (item >= A.nbatch) break;
        int g = 0;
        while (g < A.ngroups - 1 && item >= fresh_copy(A.groups + g).item_end) ++g;
        const GroupDev G = fresh_copy(A.groups + g);
        int i, j;
        tile_pixel(G.tiles_x, A.tile_w, item - G.item_begin, lane, i, j);
        const bool valid = i < G.cam.nx && j < G.cam.ny;
        const int pix = j * G.cam.nx + i;
        double alpha, beta, hlast, y[7];
        uint8_t st;
        int n;
        const int nch_w = geodesic_phase<true, kMode == kModeF32>(BatchSource{base, g, -1}, valid, i, j, slot,
                                                                  wchunks, wave, lane, alpha, beta, y, hlast, st, n);
        for (int q = G.inst_begin; q < G.inst_end; ++q)
            trace_transfer<kMode>(BatchSource{base, g, q}, slot, wchunks, lane, valid, pix, alpha, beta, st, n);
        if (lane == 0)
            for (int k = 0; k < nch_w; ++k) atomicExch(&base().chunk_flags[wchunks[k]], 0u);
    }
}

// Rays longer than the wave-synchronous store: one ray per lane with a
// full-length private store (64 B per point, the FP32-operator mode's points
// at its 32 B stride); lanes loop over the overflow list
// (entries of batch instances carry their instance).
template <int kMode>
__global__ __launch_bounds__(64) void trace_long(TraceArgs A) {
    __shared__ float s_btab_f[kMode == kModeF32 ? kBesPanels * 2 * kBesCoef : 1];
    if (kMode == kModeF32) {
        for (int k = threadIdx.x; k < kBesPanels * 2 * kBesCoef; k += blockDim.x)
            s_btab_f[k] = (float)A.btab[k];
        __syncthreads();
        A.btab_f = s_btab_f;
    }
    const unsigned total = *A.overflow_count;
    const unsigned tid = blockIdx.x * blockDim.x + threadIdx.x;
    const unsigned stride = gridDim.x * blockDim.x;
    double* path = A.long_pool + (size_t)tid * (size_t)(A.max_steps + 1) * kPointDoubles;
    for (unsigned k = tid; k < total; k += stride) {
        TraceArgs R = A;
        if (A.overflow_inst) {
            const int q = A.overflow_inst[k];
            const InstDev& I = A.inst[q];
            apply_group(R, A.groups[I.group]);
            apply_instance(R, I, q);
        }
        const int pix = A.overflow_list[k];
        const int i = pix % R.cam.nx, j = pix / R.cam.nx;
        double alpha, beta, y[7];
        // the parameters can differ from lane to lane here (batch instances),
        // so they stay in vector registers (read once per ray)
        const CameraDesc C = R.cam;
        pixel_position(C, i, j, alpha, beta);
        {
            double X[4], K[4];
            camera_launch(C, alpha, beta, X, K);
            y[0] = X[1]; y[1] = X[2]; y[2] = X[3];
            y[3] = K[0]; y[4] = K[1]; y[5] = K[2]; y[6] = K[3];
        }
        constexpr int kS = kPointStride<kMode>;
        if constexpr (kMode == kModeF32)
            store_point_f32(path, y, 0.0);
        else
            store_point(path, y, 0.0);
        double sn, cs;
        sincos_polar(y[1], sn, cs);
        uint8_t st = kRunning;
        int n = 0;
        while (st == kRunning) {
            const double h = rk4_step(R.cam.a, R.cam.m, R.eps, y, sn, cs);
            ++n;
            if constexpr (kMode == kModeF32)
                store_point_f32(path + (size_t)n * kS, y, h);
            else
                store_point(path + (size_t)n * kS, y, h);
            st = stop_test(R, y, h, n, sn);
        }
        const int n_end = (st == kNonFinite || st == kAxis) ? n - 1 : n;
        typename std::conditional<kMode == kModeF32, XferStateF, XferState>::type xs;
        Coh N;
        unsigned n_exact = 0;
        for (int m = n_end; m >= 0; --m) {
            if constexpr (kMode == kModeF32) {
                PointF pf;
                load_point_f32(path + (size_t)m * kS, pf);
                transfer_point_f32(R, pf, m, m == n_end, xs, N);
            } else {
                double pt[kPointDoubles];
                load_point(path + (size_t)m * kS, pt);
                if constexpr (kKappa<kMode>)
                    transfer_point_kappa(R, pt, m, m == n_end, xs, N, nullptr, false, n_exact);
                else
                    transfer_point(R, pt, m, m == n_end, xs, N);
            }
        }
        if constexpr (kKappa<kMode>) atomicAdd(&A.counters[9], (unsigned long long)n_exact);
        double S[4];
        camera_output(R, alpha, beta, N, S);
        const uint8_t st_out = write_pixel(R, pix, S, st, n);
        // the wave-synchronous pass counted this ray as overflow; count it now
        atomicAdd(&A.counters[0], (unsigned long long)n);
        atomicAdd(&A.counters[1 + st_out], 1ULL);
        atomicMax(&A.counters[6], (unsigned long long)n);
    }
}

// ---------------------------------------------------------------------------
// Bessel-ratio table: values at Chebyshev nodes by the trapezoid rule, then
// coefficients.  vals: [panel][node][2].
// ---------------------------------------------------------------------------
KRT_HD double scaled_bessel_k(double nu, double x) {
    // int_0^T exp(-x (cosh s - 1)) cosh(nu s) ds, trapezoid with step h; T from
    // x (cosh T - 1) - nu T >= 45, h = min(0.1, 0.5 / sqrt(x)).
    double T = 1.0;
    for (int it = 0; it < 6; ++it) T = acosh(1.0 + (45.0 + nu * T) / x);
    const double h = fmin(0.1, 0.5 / sqrt(x));
    const int ns = (int)ceil(T / h);
    double sum = 0.5;  // s = 0 term (weight 1/2)
    for (int k = 1; k <= ns; ++k) {
        const double s = k * h;
        sum += exp(-x * (cosh(s) - 1.0)) * cosh(nu * s);
    }
    return sum * h;
}

__global__ void bessel_table_nodes(double* vals) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= kBesPanels * kBesCoef) return;
    const int p = idx / kBesCoef, k = idx % kBesCoef;
    const double z = cos(kPi * (k + 0.5) / kBesCoef);
    const double x = bessel_panel_x(p, z);
    const double k0 = scaled_bessel_k(0.0, x), k1 = scaled_bessel_k(1.0, x), k2 = scaled_bessel_k(2.0, x);
    vals[idx * 2 + 0] = k0 / k2;
    vals[idx * 2 + 1] = k1 / k2;
}

__global__ void bessel_table_coefs(const double* vals, double* table) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= kBesPanels * 2 * kBesCoef) return;
    const int p = idx / (2 * kBesCoef), f = (idx / kBesCoef) % 2, j = idx % kBesCoef;
    double s = 0.0;
    for (int k = 0; k < kBesCoef; ++k)
        s += vals[(p * kBesCoef + k) * 2 + f] * cos(kPi * j * (k + 0.5) / kBesCoef);
    s *= 2.0 / kBesCoef;
    if (j == 0) s *= 0.5;
    table[(size_t)p * 2 * kBesCoef + f * kBesCoef + j] = s;
}

// Chebyshev coefficients of each (panel, function) series to monomial
// coefficients in z, in place: T_0 = 1, T_1 = z, T_(j+1) = 2 z T_j - T_(j-1)
// (integer coefficients, exact in FP64), a_i = sum_j c_j [z^i] T_j.
__global__ void bessel_table_monomial(double* table) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= kBesPanels * 2) return;
    double* c = table + (size_t)idx * kBesCoef;
    double a[kBesCoef], tp[kBesCoef], tc[kBesCoef];
    for (int i = 0; i < kBesCoef; ++i) {
        tp[i] = (i == 0) ? 1.0 : 0.0;
        tc[i] = (i == 1) ? 1.0 : 0.0;
        a[i] = c[0] * tp[i] + c[1] * tc[i];
    }
    for (int j = 2; j < kBesCoef; ++j) {
        double tn[kBesCoef];
        tn[0] = -tp[0];
        for (int i = 1; i < kBesCoef; ++i) tn[i] = 2.0 * tc[i - 1] - tp[i];
        for (int i = 0; i < kBesCoef; ++i) {
            a[i] += c[j] * tn[i];
            tp[i] = tc[i];
            tc[i] = tn[i];
        }
    }
    for (int i = 0; i < kBesCoef; ++i) c[i] = a[i];
}

// MKS inversion table: x2 at theta_k = k pi / kX2Tab for hslope h, each node
// by Newton from theta_k / pi to convergence (the start values of the
// per-point inversion in the snapshot model).
__global__ void mks_x2_table(double h, double* tab) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k > kX2Tab) return;
    const double th = k * (kPi / kX2Tab);
    const double hh = 0.5 * (1.0 - h);
    double x2 = th * (1.0 / kPi);
    for (int it = 0; it < 64; ++it) {
        double sn, cs;
        sincos_2pi(x2, sn, cs);
        const double dx = (kPi * x2 + hh * sn - th) / (kPi * (1.0 + (1.0 - h) * cs));
        x2 -= dx;
        if (fabs(dx) < 1e-16) break;
    }
    tab[k] = x2;
}

// ---------------------------------------------------------------------------
// Snapshot layout 1 ([8][ncell], one array per field) to layout 0
// ([ncell][8], the fields of a cell together, which the gather reads as
// vectors): 64 cells per block staged through LDS, so that both the reads of
// each field and the writes of whole cells are coalesced.
// ---------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(256) void snapshot_to_cells(const T* __restrict__ src, T* __restrict__ dst,
                                                         size_t ncell) {
    __shared__ T tile[8][65];
    const size_t c0 = (size_t)blockIdx.x * 64;
    const int lane = threadIdx.x & 63, grp = threadIdx.x >> 6;   // 4 groups of 64 threads
    for (int q = grp; q < 8; q += 4) {
        const size_t c = c0 + lane;
        tile[q][lane] = c < ncell ? src[(size_t)q * ncell + c] : T(0);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < 512; k += 256) {
        const size_t c = c0 + k / 8;
        if (c < ncell) dst[c * 8 + (k % 8)] = tile[k % 8][k / 8];
    }
}

// ---------------------------------------------------------------------------
// Image reduction: per-block compensated partial sums of the four Stokes
// planes and the maximum of I, then one block combining them.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void neumaier_add(double& s, double& c, double x) {
    const double t = s + x;
    if (fabs(s) >= fabs(x)) c += (s - t) + x;
    else c += (x - t) + s;
    s = t;
}

__global__ __launch_bounds__(256) void reduce_partial(const double* __restrict__ stokes, size_t np,
                                                      double* partial) {
    __shared__ double sh[256 * 9];
    double s[4] = {0, 0, 0, 0}, c[4] = {0, 0, 0, 0}, mx = -INFINITY;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < np;
         k += (size_t)gridDim.x * blockDim.x) {
        for (int q = 0; q < 4; ++q) neumaier_add(s[q], c[q], stokes[q * np + k]);
        mx = fmax(mx, stokes[k]);
    }
    for (int q = 0; q < 4; ++q) {
        sh[threadIdx.x * 9 + 2 * q] = s[q];
        sh[threadIdx.x * 9 + 2 * q + 1] = c[q];
    }
    sh[threadIdx.x * 9 + 8] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        double S[4] = {0, 0, 0, 0}, Cc[4] = {0, 0, 0, 0}, M = -INFINITY;
        for (int t = 0; t < (int)blockDim.x; ++t) {
            for (int q = 0; q < 4; ++q) {
                neumaier_add(S[q], Cc[q], sh[t * 9 + 2 * q]);
                Cc[q] += sh[t * 9 + 2 * q + 1];
            }
            M = fmax(M, sh[t * 9 + 8]);
        }
        for (int q = 0; q < 4; ++q) {
            partial[blockIdx.x * 9 + 2 * q] = S[q];
            partial[blockIdx.x * 9 + 2 * q + 1] = Cc[q];
        }
        partial[blockIdx.x * 9 + 8] = M;
    }
}

__global__ void reduce_final(const double* partial, int nblocks, double scale, double* out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double S[4] = {0, 0, 0, 0}, Cc[4] = {0, 0, 0, 0}, M = -INFINITY;
    for (int b = 0; b < nblocks; ++b) {
        for (int q = 0; q < 4; ++q) {
            neumaier_add(S[q], Cc[q], partial[b * 9 + 2 * q]);
            Cc[q] += partial[b * 9 + 2 * q + 1];
        }
        M = fmax(M, partial[b * 9 + 8]);
    }
    for (int q = 0; q < 4; ++q) out[q] = scale * (S[q] + Cc[q]);
    out[4] = M;
}

// ---------------------------------------------------------------------------
// Component hooks.
// ---------------------------------------------------------------------------
__global__ void hook_plasma(TraceArgs A, int64_t n, double a, double m, const double* X,
                            double* out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double r = X[k * 3], th = X[k * 3 + 1], ph = X[k * 3 + 2];
    Metric g;
    metric_eval(a, m, r, th, g);
    Plasma p{};
    // the model itself (plasma_at also skips points the transfer leaves alone)
    const bool ok = A.model == kModelSnapshot ? snapshot_plasma(A.snap, a, m, r, th, ph, g, p) == 1
                                              : adaf_plasma(A.adaf, a, m, r, g, p);
    double* o = out + k * 12;
    o[0] = p.ne; o[1] = p.thetae; o[2] = p.B;
    for (int q = 0; q < 4; ++q) {
        o[3 + q] = ok ? p.u[q] : 0.0;
        o[7 + q] = ok ? p.b[q] : 0.0;
    }
    o[11] = ok ? 1.0 : 0.0;
}

__global__ void hook_coeffs(const double* btab, int64_t n, const double* in, double* out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double* v = in + k * 5;
    double c[8];
    thermal_coefficients(btab, v[0], v[1], v[2], v[3], v[4], c);
    for (int q = 0; q < 8; ++q) out[k * 8 + q] = c[q];
}

// FP64 FMA issue probe: each thread advances `kChains` independent FMA chains
// iters x 16 steps; thread 0 of a block writes its sum (the chains stay live).
template <int kChains>
__global__ __launch_bounds__(256) void fma_probe(double* out, int iters, double x, double y) {
    double a[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) a[c] = 1e-3 * (double)threadIdx.x + (double)c;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < 16; ++u)
#pragma unroll
            for (int c = 0; c < kChains; ++c) a[c] = fma(a[c], x, y);
    }
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += a[c];
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

__global__ void hook_bessel(const double* btab, int64_t n, const double* x, double* out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double a, b;
    bessel_ratios(btab, x[k], a, b);
    out[2 * k] = a;
    out[2 * k + 1] = b;
}

__global__ void hook_mueller(int64_t n, const double* coef, const double* S, double w, double* out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double* c = coef + k * 6;
    double s[4] = {S[k * 4], S[k * 4 + 1], S[k * 4 + 2], S[k * 4 + 3]};
    mueller_thermal(c[0], c[1], c[2], c[3], c[4], c[5], w, s);
    for (int q = 0; q < 4; ++q) out[k * 4 + q] = s[q];
}

__global__ void hook_mueller_general(int64_t n, const double* coef, const double* S, double w, double* out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double* c = coef + k * 8;
    double s[4] = {S[k * 4], S[k * 4 + 1], S[k * 4 + 2], S[k * 4 + 3]};
    mueller_general(c[0], c[1], c[2], c[3], c[4], c[5], c[6], c[7], w, s);
    for (int q = 0; q < 4; ++q) out[k * 4 + q] = s[q];
}

__global__ void hook_kappa_integrals(const double* syntab, int64_t n, const double* in, double* out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double o[8];
    kappa_integrals(syntab, in[k * 3], in[k * 3 + 1], in[k * 3 + 2], o);
    for (int q = 0; q < 8; ++q) out[k * 8 + q] = o[q];
}

}  // namespace krt
