/*
 * Plasma models evaluated at a point of the stored geodesic.
 * Test infrastructure only (CPU oracle).
 *
 * Sec. 2.1: plasma quantities are needed at every step of the transfer
 * integration, either computed along the ray for a semianalytic ADAF model or
 * interpolated from precomputed 3D GRMHD arrays.  Neither model's parameters
 * are given; readings:
 *
 * ADAF: n_e = n0 r^-3/2 exp(-z^2 / (2 (h r)^2)) with z = r cos(theta);
 *   T_e = T0 / r; Keplerian angular velocity Omega = 1/(r^3/2 + a) outside
 *   the ISCO, the zero-angular-momentum observer inside it (or where the
 *   Keplerian velocity is not timelike); |B| from beta = p_virial / p_mag
 *   with p_virial = n_e m_p c^2 / (6 r); toroidal field
 *   b^mu = |B| (delta^mu_phi + u_phi u^mu) / sqrt(g_phph + u_phi^2).
 *
 * Snapshot: modified Kerr-Schild grid x1 = ln r, theta = pi x2 +
 *   (1-h)/2 sin(2 pi x2), x3 = phi, cell-centred trilinear interpolation of
 *   the primitives (rho, u, U1..3, B1..3), then the four-velocity from the
 *   velocity relative to normal observers and b^mu from B^i; electron
 *   temperature from the R_high / R_low prescription; no emission where
 *   b.b/rho > sigma_cut or r > r_emit_max.
 *
 * Flat-space test models: a static ball of uniform plasma with a uniform
 * field (Cartesian direction), or a ball of given invariant coefficients.
 */
#include <cmath>
#include "oracle_internal.h"

namespace orc {

static void zamo_or_kepler(double a, double m, double r, double th, bool kepler, double u[4]) {
    Mat4 g;
    metric(a, m, r, th, g);
    u[0] = u[1] = u[2] = u[3] = 0.0;
    double Om = 0.0, norm = 1.0;
    if (kepler) {
        Om = 1.0 / (std::pow(r, 1.5) + a);
        norm = g[0][0] + 2.0 * g[0][3] * Om + g[3][3] * Om * Om;
    }
    if (!kepler || !(norm < 0.0)) {
        Om = -g[0][3] / g[3][3];
        norm = g[0][0] + 2.0 * g[0][3] * Om + g[3][3] * Om * Om;
    }
    if (!(norm < 0.0)) {
        u[0] = NAN;
        return;
    }
    u[0] = 1.0 / std::sqrt(-norm);
    u[3] = Om * u[0];
}

static int adaf(const or_model* md, double a, double m, double r, double th, Plasma* p) {
    double z = r * std::cos(th);
    double H = md->h_over_r * r;
    p->ne = md->n0_cgs * std::pow(r, -1.5) * std::exp(-z * z / (2.0 * H * H));
    double Te = md->T0_K / r;
    p->thetae = K_BOLTZ * Te / (M_ELECTRON * C_LIGHT * C_LIGHT);
    double B2 = 8.0 * PI * p->ne * M_PROTON * C_LIGHT * C_LIGHT / (6.0 * r * md->beta);
    p->B = std::sqrt(B2);
    bool kepler = (m != 0.0) && (r >= isco(a));
    zamo_or_kepler(a, m, r, th, kepler, p->u);
    if (!std::isfinite(p->u[0])) return 0;
    Mat4 g;
    metric(a, m, r, th, g);
    double ul[4];
    lower(g, p->u, ul);
    double nb = std::sqrt(g[3][3] + ul[3] * ul[3]);
    for (int mu = 0; mu < 4; ++mu) p->b[mu] = p->B * ((mu == 3 ? 1.0 : 0.0) + ul[3] * p->u[mu]) / nb;
    return 1;
}

/* Cartesian vector -> contravariant components in flat spherical coordinates. */
static void cartesian_to_spherical(const double v[3], double r, double th, double ph, double out[4]) {
    double st = std::sin(th), ct = std::cos(th), sp = std::sin(ph), cp = std::cos(ph);
    out[0] = 0.0;
    out[1] = v[0] * st * cp + v[1] * st * sp + v[2] * ct;
    out[2] = (v[0] * ct * cp + v[1] * ct * sp - v[2] * st) / r;
    out[3] = (-v[0] * sp + v[1] * cp) / (r * st);
}

static int slab(const or_model* md, double r, double th, double ph, Plasma* p) {
    bool inside = r < md->slab_radius;
    p->ne = inside ? md->slab_ne : 0.0;
    p->thetae = md->slab_thetae;
    p->B = md->slab_B;
    p->u[0] = 1.0;
    p->u[1] = p->u[2] = p->u[3] = 0.0;
    double bd[3] = {md->slab_bdir[0], md->slab_bdir[1], md->slab_bdir[2]};
    double nb = std::sqrt(bd[0] * bd[0] + bd[1] * bd[1] + bd[2] * bd[2]);
    double v[3] = {p->B * bd[0] / nb, p->B * bd[1] / nb, p->B * bd[2] / nb};
    cartesian_to_spherical(v, r, th, ph, p->b);
    return 1;
}

/* ---- snapshot ---- */

/* theta(x2) of the modified Kerr-Schild grid and its derivative. */
static double mks_theta(double x2, double h) { return PI * x2 + 0.5 * (1.0 - h) * std::sin(2.0 * PI * x2); }
static double mks_dtheta(double x2, double h) { return PI * (1.0 + (1.0 - h) * std::cos(2.0 * PI * x2)); }

/* Trilinear interpolation of the 8 primitives at grid coordinates
 * (x1, x2, x3), cell-centred; clamp to the end cells in x1 and x2,
 * periodic in x3. */
static void interp_prims(const or_snapshot* s, double x1, double x2, double x3, double P[8]) {
    double X[3] = {(x1 - s->x1_start) / s->dx1 - 0.5, (x2 - s->x2_start) / s->dx2 - 0.5,
                   (x3 - s->x3_start) / s->dx3 - 0.5};
    int n[3] = {s->n1, s->n2, s->n3};
    int i0[3], i1[3];
    double d[3];
    for (int k = 0; k < 2; ++k) {
        double f = std::floor(X[k]);
        int i = (int)f;
        double t = X[k] - f;
        if (i < 0) { i = 0; t = 0.0; }
        if (i > n[k] - 2) { i = n[k] - 2; t = 1.0; }
        if (n[k] == 1) { i = 0; t = 0.0; }
        i0[k] = i;
        i1[k] = (n[k] == 1) ? 0 : i + 1;
        d[k] = t;
    }
    {
        double f = std::floor(X[2]);
        double t = X[2] - f;
        long i = (long)f;
        long nn = n[2];
        long a0 = ((i % nn) + nn) % nn;
        i0[2] = (int)a0;
        i1[2] = (int)((a0 + 1) % nn);
        d[2] = t;
    }
    for (int q = 0; q < 8; ++q) P[q] = 0.0;
    for (int c = 0; c < 8; ++c) {
        int ia = (c & 4) ? i1[0] : i0[0];
        int ib = (c & 2) ? i1[1] : i0[1];
        int ic = (c & 1) ? i1[2] : i0[2];
        double w = ((c & 4) ? d[0] : 1.0 - d[0]) * ((c & 2) ? d[1] : 1.0 - d[1]) *
                   ((c & 1) ? d[2] : 1.0 - d[2]);
        const double* cell = s->prims + 8 * (((size_t)ia * s->n2 + ib) * s->n3 + ic);
        for (int q = 0; q < 8; ++q) P[q] += w * cell[q];
    }
}

static int snapshot(const or_snapshot* s, double a, double m, double r, double th, double ph,
                    double L_cm, Plasma* p) {
    /* grid coordinates: x1 = ln r, invert theta(x2) by 8 Newton steps from theta/pi */
    double x1 = std::log(r);
    double x2 = th / PI;
    for (int it = 0; it < 8; ++it) x2 -= (mks_theta(x2, s->hslope) - th) / mks_dtheta(x2, s->hslope);
    double x3 = ph;
    double P[8];
    interp_prims(s, x1, x2, x3, P);
    double rho = P[0], uu = P[1];
    /* a non-finite value among the gathered primitives where the snapshot
     * emits: reported (2), and the transfer poisons the ray with it */
    if (r <= s->r_emit_max && !std::isfinite(P[0] + P[1] + P[2] + P[3] + P[4] + P[5] + P[6] + P[7]))
        return 2;

    /* metric in grid coordinates: g_mks = J^T g_ks J, J = diag(1, r, dtheta/dx2, 1) */
    Mat4 gks, g, gi;
    metric(a, m, r, th, gks);
    double J[4] = {1.0, r, mks_dtheta(x2, s->hslope), 1.0};
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) g[i][j] = gks[i][j] * J[i] * J[j];
    invert4(g, gi);
    /* four-velocity from the velocity relative to normal observers:
     * u^t = gamma / lapse, u^i = U^i - gamma lapse g^{ti} */
    double lapse = 1.0 / std::sqrt(-gi[0][0]);
    double ut3[3] = {P[2], P[3], P[4]};
    double qsum = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) qsum += g[i + 1][j + 1] * ut3[i] * ut3[j];
    double gamma = std::sqrt(1.0 + qsum);
    double u[4];
    u[0] = gamma / lapse;
    for (int i = 0; i < 3; ++i) u[i + 1] = ut3[i] - gamma * lapse * gi[0][i + 1];
    /* field four-vector: b^t = B^i u_i, b^i = (B^i + b^t u^i) / u^t */
    double ul[4];
    lower(g, u, ul);
    double Bv[3] = {P[5], P[6], P[7]};
    double b[4];
    b[0] = Bv[0] * ul[1] + Bv[1] * ul[2] + Bv[2] * ul[3];
    for (int i = 0; i < 3; ++i) b[i + 1] = (Bv[i] + b[0] * u[i + 1]) / u[0];
    double bsq = dot(g, b, b);

    /* back to Kerr-Schild components */
    for (int mu = 0; mu < 4; ++mu) {
        p->u[mu] = u[mu] * J[mu];
        p->b[mu] = b[mu] * J[mu];
    }

    /* code units -> cgs */
    double rho_unit = s->M_unit_g / (L_cm * L_cm * L_cm);
    double B_unit = C_LIGHT * std::sqrt(4.0 * PI * rho_unit);
    p->B = std::sqrt(bsq > 0.0 ? bsq : 0.0) * B_unit;
    p->ne = rho * rho_unit / (M_PROTON + M_ELECTRON);
    /* R_high / R_low electron temperature: T_i/T_e = (R_high beta^2 + R_low)/(1 + beta^2),
     * beta = (gamma_ad - 1) u / (b.b / 2); written with 1/beta^2 so that b = 0 gives R_high */
    double thetae = 0.0;
    if (rho > 0.0 && uu > 0.0) {
        double ib = 0.5 * bsq / ((s->gamma_ad - 1.0) * uu);
        double ib2 = ib * ib;
        double trat = (s->R_high + s->R_low * ib2) / (1.0 + ib2);
        thetae = (M_PROTON / M_ELECTRON) * (s->gamma_ad - 1.0) * (uu / rho) / (1.0 + trat);
    }
    p->thetae = thetae;
    if (!(rho > 0.0) || bsq / rho > s->sigma_cut || r > s->r_emit_max) p->ne = 0.0;
    return 1;
}

int plasma(const or_model* model, const or_snapshot* snap, double a, double m,
           double r, double th, double ph, double L_cm, Plasma* p) {
    switch (model->kind) {
        case OR_MODEL_ADAF: return adaf(model, a, m, r, th, p);
        case OR_MODEL_SLAB_PLASMA:
        case OR_MODEL_SLAB_FIXED: return slab(model, r, th, ph, p);
        case OR_MODEL_SNAPSHOT: return snapshot(snap, a, m, r, th, ph, L_cm, p);
        default: return 0;
    }
}

int validate_model(const or_model* model, const or_snapshot* snap, const or_camera* cam) {
    if (!model) return -1;
    switch (model->kind) {
        case OR_MODEL_ADAF:
            if (!(model->n0_cgs >= 0.0) || !(model->T0_K > 0.0) || !(model->beta > 0.0) ||
                !(model->h_over_r > 0.0))
                return -1;
            return 0;
        case OR_MODEL_SLAB_PLASMA:
        case OR_MODEL_SLAB_FIXED:
            /* flat space, spherical coordinates only */
            if (cam->mass_factor != 0 || cam->a != 0.0) return -1;
            return 0;
        case OR_MODEL_SNAPSHOT:
            if (!snap || !snap->prims || snap->n1 < 2 || snap->n2 < 2 || snap->n3 < 1) return -1;
            if (!(snap->dx1 > 0.0 && snap->dx2 > 0.0 && snap->dx3 > 0.0)) return -1;
            if (!(snap->M_unit_g > 0.0) || !(snap->gamma_ad > 1.0)) return -1;
            return 0;
        default:
            return -1;
    }
}

}  // namespace orc

extern "C" int or_plasma(const or_model* model, const or_snapshot* snap, double a, double m,
                         double r, double th, double ph, double L_cm, double out[11]) {
    orc::Plasma p;
    int ok = orc::plasma(model, snap, a, m, r, th, ph, L_cm, &p);
    out[0] = p.ne;
    out[1] = p.thetae;
    out[2] = p.B;
    for (int k = 0; k < 4; ++k) {
        out[3 + k] = p.u[k];
        out[7 + k] = p.b[k];
    }
    return ok;
}
